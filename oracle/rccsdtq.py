"""Spin-restricted CCSDTQ on full spin-free tensors, FP64 (test oracle only).

Test infrastructure: only tests and the benchmark's CPU baseline use this
module; the HIP library never does.

Follows the paper's Appendix "RCCSDTQ" on top of the RCCSDT oracle
(oracle.rccsdt): the quadruples-driven term of the doubles residual, the T4
corrections of the triples residual, the quadruples residual (Eq.
resi-rccsdtq) with its intermediates, the spin summations of Eq.
quadruples-spin-sum, and the R4 post-processing of Sec. "Removing
redundancies in RCC amplitudes" (symmetrization of blocks with two equal
occupied indices, purification of blocks with three or more, and the
projection Eq. T4ortho onto the 14-dimensional non-redundant subspace of the
24 virtual permutations).

Readings (as for RCCSDT): index placement X_{lower}^{upper} is the tensor
X^{upper}_{lower}; v[p,q,r,s] = v^{pq}_{rs}; f~_e^m is row m, column e of the
dressed Fock matrix; a check on an integral column is
v^{p'q}_{r's} = 2 v^{pq}_{rs} - v^{pq}_{sr}; a check on amplitude columns acts
on the virtual labels of the written tensor with the occupied ones fixed;
P_{(x)(y)..} is the unnormalised sum over the simultaneous permutations of
the listed columns.  Array convention t4[i,j,k,l,a,b,c,d].
"""

from __future__ import annotations

import itertools

import numpy as np

from . import rccsdt as R

PERMS4 = list(itertools.permutations(range(4)))


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def _swapv(x, p, q):
    """Exchange virtual positions p and q (0..3) of an [o,o,o,o,v,v,v,v] tensor."""
    ax = list(range(8))
    ax[4 + p], ax[4 + q] = ax[4 + q], ax[4 + p]
    return x.transpose(ax)


def chk4_1(t4):
    """Single check on column 1 (Eq. quadruples-spin-sum):
    (2 - P_a^b - P_a^c - P_a^d) t^{abcd}."""
    return 2.0 * t4 - _swapv(t4, 0, 1) - _swapv(t4, 0, 2) - _swapv(t4, 0, 3)


def chk4_12(t4):
    """Double check on columns 1, 2: (2 - P_b^c - P_b^d) applied to chk4_1."""
    s = chk4_1(t4)
    return 2.0 * s - _swapv(s, 1, 2) - _swapv(s, 1, 3)


def perm_sym4(X):
    """P_{(ia)(jb)(kc)(ld)}: sum over the 24 simultaneous column permutations."""
    out = np.zeros_like(X)
    for p in PERMS4:
        out += X.transpose(*p, *(4 + q for q in p))
    return out


# ---------------------------------------------------------------------------
# Intermediates of the RCCSDTQ appendix
# ---------------------------------------------------------------------------

def rccsdtq_intermediates(ft, Vt, t2, t3, t4, o, ims, ims3):
    """Wbar_ej^ab, W_iej^mab, W_ijk^amn, W_eij^mab, W_ejk^abc, W_ijk^abm and
    Wtilde_ei^ma as arrays with the lower indices first, then the upper ones
    (e.g. Wiej[i,e,j,m,a,b] = W_iej^mab)."""
    n = ft.shape[0]
    O, Vs = slice(0, o), slice(o, n)
    Vc = R.vchk(Vt)
    tau = R.chk2(t2)
    s1_3 = R.chk3_1(t3)
    s1_4 = chk4_1(t4)
    fov = ft[O, Vs]
    # Wbar_ej^ab = W_ej^ab - sum_m f~_e^m t_mj^ab, as Wbej[a,b,e,j]
    Wbej = ims3["Wvvvo"] - _es("me,mjab->abej", fov, t2)
    # W_iej^mab = sum_f v^{ma}_{fe} t_ji^bf - sum_n v^{mn}_{ie} t_nj^ab - 1/2 sum_fn v^{nm}_{ef} t_inj^fab
    Wiej = (_es("mafe,jibf->iejmab", Vt[O, Vs, Vs, Vs], t2)
            - _es("mnie,njab->iejmab", Vt[O, O, O, Vs], t2)
            - 0.5 * _es("nmef,injfab->iejmab", Vt[O, O, Vs, Vs], t3))
    # W_ijk^amn = P_(mj)(nk) [ sum_e v^{mn}_{ek} t_ij^ae + 1/2 sum_ef v^{mn}_{ef} t_ijk^aef ]
    g = (_es("mnek,ijae->ijkamn", Vt[O, O, Vs, O], t2)
         + 0.5 * _es("mnef,ijkaef->ijkamn", Vt[O, O, Vs, Vs], t3))
    Wijk_amn = g + g.transpose(0, 2, 1, 3, 5, 4)
    # W_eij^mab = P_(ia)(jb) [ sum_f v^{m'a}_{e'f} t_ji^bf - sum_n v^{m'n}_{e'i} t_nj^ab
    #                          + 1/4 sum_fn v^{n'm}_{f'e} t_{n'ij}^{f'ab} ]
    g = (_es("maef,jibf->eijmab", Vc[O, Vs, Vs, Vs], t2)
         - _es("mnei,njab->eijmab", Vc[O, O, Vs, O], t2)
         + 0.25 * _es("nmfe,nijfab->eijmab", Vc[O, O, Vs, Vs], s1_3))
    Weij = g + g.transpose(0, 2, 1, 3, 5, 4)
    # W_ejk^abc = P_(jb)(kc) [ 1/2 sum_f W_ef^ab t_jk^fc - 1/2 sum_fmn v^{mn}_{ef} t_{n'mjk}^{f'abc} ]
    g = (0.5 * _es("abef,jkfc->ejkabc", ims3["Wvvvv"], t2)
         - 0.5 * _es("mnef,nmjkfabc->ejkabc", Vt[O, O, Vs, Vs], s1_4))
    Wejk = g + g.transpose(0, 2, 1, 3, 5, 4)
    # Wtilde_ei^ma = v^{ma}_{ei} + 1/2 sum_nf v^{n'm}_{f'e} t_{n'i}^{f'a} - 1/2 sum_nf v^{nm}_{ef} t_in^fa
    Wt_ei = (Vt[O, Vs, Vs, O].transpose(2, 3, 0, 1)
             + 0.5 * _es("nmfe,nifa->eima", Vc[O, O, Vs, Vs], tau)
             - 0.5 * _es("nmef,infa->eima", Vt[O, O, Vs, Vs], t2))
    # W_ijk^abm = P_(ia)(jb) [ sum_ef v^{am}_{ef} t_ijk^ebf + sum_e Wtilde_ei^ma t_jk^be
    #   + sum_e W_ke^ma t_ji^be - 1/2 sum_n W_ki^mn t_nj^ab + 1/2 sum_efn v^{mn}_{ef} t_{n'ijk}^{f'abe} ]
    # W_ke^ma here is the barred intermediate Wbar^{ma}_{ke} of the RCCSDT
    # appendix (the reading the brute-force residual fixes; the RCCSD
    # W^{ma}_{ke} leaves a discrepancy cubic in T2)
    g = (_es("amef,ijkebf->ijkabm", Vt[Vs, O, Vs, Vs], t3)
         + _es("eima,jkbe->ijkabm", Wt_ei, t2)
         + _es("make,jibe->ijkabm", ims3["Wbar_ovov"], t2)
         - 0.5 * _es("mnki,njab->ijkabm", ims["Woooo"], t2)
         + 0.5 * _es("mnef,nijkfabe->ijkabm", Vt[O, O, Vs, Vs], s1_4))
    Wijk_abm = g + g.transpose(1, 0, 2, 4, 3, 5)
    return dict(Wbej=Wbej, Wiej=Wiej, Wijk_amn=Wijk_amn, Weij=Weij, Wejk=Wejk, Wt_ei=Wt_ei, Wijk_abm=Wijk_abm)


R4_TERMS = ("T3_WBAR", "T3_WVOOO", "F_VV", "F_OO", "RING_A", "RING_B", "RING_C", "HH", "PP",
            "W_EIJ", "W_IEJ_1", "W_IEJ_2", "W_IJK_AMN", "W_IJK_ABM", "W_EJK")


def pp_term(W, t4):
    """The particle-particle ladder term of Eq. resi-rccsdtq before the
    permutation operator: 1/4 sum_ef W^{ab}_{ef} t_ijkl^efcd, W[a,b,e,f]."""
    return 0.25 * _es("abef,ijklefcd->ijklabcd", W, t4)


def r4_terms(t2, t3, t4, ims, ims3, ims4):
    """The fifteen terms inside P_{(ia)(jb)(kc)(ld)} of Eq. resi-rccsdtq, in
    the order written there, as [o,o,o,o,v,v,v,v] tensors."""
    s1_3 = R.chk3_1(t3)
    s1_4 = chk4_1(t4)
    return {
        "T3_WBAR": 0.5 * _es("abej,iklecd->ijklabcd", ims4["Wbej"], t3),
        "T3_WVOOO": -0.5 * _es("amij,mklbcd->ijklabcd", ims3["Wvooo"], t3),
        "F_VV": (1.0 / 6.0) * _es("ae,ijklebcd->ijklabcd", ims["Fvv"], t4),
        "F_OO": -(1.0 / 6.0) * _es("mi,mjklabcd->ijklabcd", ims["Foo"], t4),
        "RING_A": (1.0 / 12.0) * _es("maei,mjklebcd->ijklabcd", ims3["Wbar_ovvo"], s1_4),
        "RING_B": -0.25 * _es("maie,jmklebcd->ijklabcd", ims3["Wbar_ovov"], t4),
        "RING_C": -0.5 * _es("mbie,jmkleacd->ijklabcd", ims3["Wbar_ovov"], t4),
        "HH": 0.25 * _es("mnij,mnklabcd->ijklabcd", ims["Woooo"], t4),
        "PP": pp_term(ims3["Wvvvv"], t4),
        "W_EIJ": 0.125 * _es("eijmab,mklecd->ijklabcd", ims4["Weij"], s1_3),
        "W_IEJ_1": -0.5 * _es("iejmab,kmlecd->ijklabcd", ims4["Wiej"], t3),
        "W_IEJ_2": -_es("iejmcb,kmlead->ijklabcd", ims4["Wiej"], t3),
        "W_IJK_AMN": 0.5 * _es("ijkamn,mnlbcd->ijklabcd", ims4["Wijk_amn"], t3),
        "W_IJK_ABM": -0.5 * _es("ijkabm,mlcd->ijklabcd", ims4["Wijk_abm"], t2),
        "W_EJK": 0.5 * _es("ejkabc,iled->ijklabcd", ims4["Wejk"], t2),
    }


def residuals(f, V, t1, t2, t3, t4, o, terms=None):
    """Raw residuals (R1, R2, R3, R4) of RCCSDTQ.  R3 and R4 are returned
    before post-processing; ``terms`` optionally restricts R4 to a subset of
    R4_TERMS."""
    n = f.shape[0]
    O, Vs = slice(0, o), slice(o, n)
    r1, r2, r3 = R.residuals(f, V, t1, t2, t3, o)
    ft, Vt = R.dress(f, V, t1)
    ims = R.ccsd_intermediates(ft, Vt, t2, o)
    ims3 = R.ccsdt_intermediates(ft, Vt, t2, t3, o, ims)
    fov = ft[O, Vs]
    s1_4 = chk4_1(t4)
    # doubles: P_(ia)(jb) [ 1/4 sum_efmn v^{mn}_{ef} t_{m'n'ij}^{e'f'ab} ]
    x2 = 0.25 * _es("mnef,mnijefab->ijab", Vt[O, O, Vs, Vs], chk4_12(t4))
    r2 = r2 + x2 + x2.transpose(1, 0, 3, 2)
    # triples: P_(ia)(jb)(kc) [ 1/6 sum f~_e^m t_{m'ijk}^{e'abc} + 1/2 sum v^{am}_{ef} t_{m'ijk}^{f'ebc}
    #                           - 1/2 sum v^{mn}_{ej} t_{m'ink}^{e'abc} ]
    x3 = ((1.0 / 6.0) * _es("me,mijkeabc->ijkabc", fov, s1_4)
          + 0.5 * _es("amef,mijkfebc->ijkabc", Vt[Vs, O, Vs, Vs], s1_4)
          - 0.5 * _es("mnej,minkeabc->ijkabc", Vt[O, O, Vs, O], s1_4))
    r3 = r3 + R.perm_sym3(x3)
    ims4 = rccsdtq_intermediates(ft, Vt, t2, t3, t4, o, ims, ims3)
    use = R4_TERMS if terms is None else terms
    parts = r4_terms(t2, t3, t4, ims, ims3, ims4)
    x4 = np.zeros_like(t4)
    for name in use:
        x4 += parts[name]
    r4 = perm_sym4(x4)
    return r1, r2, r3, r4


# ---------------------------------------------------------------------------
# R4 post-processing (Sec. "Removing redundancies in RCC amplitudes")
# ---------------------------------------------------------------------------

def symmetrize_r4(r4):
    """Blocks with exactly one pair of equal neighbouring occupied indices in
    the triangular sector are averaged over the swap of the corresponding
    virtual indices: i=j<k<=l over (a,b), i<j=k<l over (b,c), i<=j<k=l over
    (c,d) (on a full tensor from the permutation operator this only removes
    roundoff).  Applied to every stored block and its column images."""
    r = r4.copy()
    o = r.shape[0]
    for i, j, k, l in itertools.product(range(o), repeat=4):
        if not (i <= j <= k <= l):
            continue
        blk = r4[i, j, k, l]
        if i == j < k <= l:
            blk = 0.5 * (blk + blk.transpose(1, 0, 2, 3))
        if i < j == k < l:
            blk = 0.5 * (blk + blk.transpose(0, 2, 1, 3))
        if i <= j < k == l:
            blk = 0.5 * (blk + blk.transpose(0, 1, 3, 2))
        r[i, j, k, l] = blk
    # the other orderings follow by the column symmetry
    out = np.empty_like(r)
    for i, j, k, l in itertools.product(range(o), repeat=4):
        occ = (i, j, k, l)
        order = sorted(range(4), key=lambda s: occ[s])
        inv = [order.index(s) for s in range(4)]
        out[i, j, k, l] = r[tuple(occ[s] for s in order)].transpose(inv)
    return out


def purify_r4(r4):
    """Zero the blocks with three or more equal occupied indices."""
    r = r4.copy()
    o = r.shape[0]
    for i, j, k, l in itertools.product(range(o), repeat=4):
        occ = (i, j, k, l)
        if max(occ.count(x) for x in occ) >= 3:
            r[i, j, k, l] = 0.0
    return r


def _chi31(p):
    """Character of the [3,1] irreducible representation of S4 at p: the
    number of fixed points minus one."""
    return sum(1 for k in range(4) if p[k] == k) - 1


def project_r4(r4):
    """(1 - Pi_[4] - Pi_[3,1]) R4 (Eq. T4ortho) with Pi_[4] = 1/24 sum_pi P_pi and
    Pi_[3,1] = 3/24 sum_pi chi_[3,1](pi) P_pi, P_pi permuting the virtual indices."""
    acc = np.zeros_like(r4)
    for p in PERMS4:
        c = (1.0 + 3.0 * _chi31(p)) / 24.0
        if c != 0.0:
            acc += c * r4.transpose(0, 1, 2, 3, *(4 + q for q in p))
    return r4 - acc


def project_r4_polynomial(r4):
    """The same projector as the polynomial in Omega (the sum of the six
    virtual transpositions) given with Eq. T4ortho:
    (Omega - 6)(Omega - 2)(2 Omega^2 + 19 Omega + 48) / 576."""
    def omega(x):
        return sum(_swapv(x, p, q) for p, q in itertools.combinations(range(4), 2))
    y = 48.0 * r4 + 19.0 * omega(r4) + 2.0 * omega(omega(r4))
    y = omega(y) - 2.0 * y
    y = omega(y) - 6.0 * y
    return y / 576.0


def postprocess_r4(r4):
    return project_r4(purify_r4(symmetrize_r4(r4)))


def denominators4(f, o):
    e = np.diag(f)
    eo, ev = e[:o], e[o:]
    occ = eo[:, None, None, None] + eo[None, :, None, None] + eo[None, None, :, None] + eo[None, None, None, :]
    vir = ev[:, None, None, None] + ev[None, :, None, None] + ev[None, None, :, None] + ev[None, None, None, :]
    return occ[:, :, :, :, None, None, None, None] - vir[None, None, None, None]


def iterate(f, V, t1, t2, t3, t4, o, diis=None):
    """One Jacobi step t += r / eps on all four ranks (R3 and R4
    post-processed), optional DIIS over the concatenated vector; returns the
    new amplitudes, the energy and the squared residual norms."""
    r1, r2, r3, r4 = residuals(f, V, t1, t2, t3, t4, o)
    r3 = R.postprocess_r3(r3)
    r4 = postprocess_r4(r4)
    d1, d2, d3 = R.denominators(f, o)
    d4 = denominators4(f, o)
    n1, n2, n3, n4 = t1 + r1 / d1, t2 + r2 / d2, t3 + r3 / d3, t4 + r4 / d4
    if diis is not None:
        new = np.concatenate([x.ravel() for x in (n1, n2, n3, n4)])
        old = np.concatenate([x.ravel() for x in (t1, t2, t3, t4)])
        out = diis.update(new, new - old)
        sizes = [x.size for x in (n1, n2, n3, n4)]
        cuts = np.cumsum(sizes)[:-1]
        n1, n2, n3, n4 = (part.reshape(x.shape) for part, x in zip(np.split(out, cuts), (n1, n2, n3, n4)))
    e = R.energy(f, V, n1, n2, o)
    norms = tuple(float(np.sum(x * x)) for x in (r1, r2, r3, r4))
    return n1, n2, n3, n4, e, norms


def solve(f, V, o, max_iter=300, tol=1e-10, diis=True):
    """Iterate from the MP2 guess (T3 = T4 = 0) until the residual norm is
    below tol; returns (energy, t1, t2, t3, t4, iterations, converged)."""
    t1, t2, t3 = R.mp2_guess(f, V, o)
    v = f.shape[0] - o
    t4 = np.zeros((o, o, o, o, v, v, v, v))
    d = R.DIIS() if diis else None
    e = R.energy(f, V, t1, t2, o)
    for it in range(1, max_iter + 1):
        t1, t2, t3, t4, e, nrm = iterate(f, V, t1, t2, t3, t4, o, diis=d)
        if np.sqrt(sum(nrm)) < tol:
            return e, t1, t2, t3, t4, it, True
    return e, t1, t2, t3, t4, max_iter, False


# ---------------------------------------------------------------------------
# Packed (i <= j <= k <= l) storage
# ---------------------------------------------------------------------------

def packed_list4(o):
    """Occupied quadruples i <= j <= k <= l in lexicographic order."""
    return [q for q in itertools.product(range(o), repeat=4) if q[0] <= q[1] <= q[2] <= q[3]]


def pack_t4(t4):
    return np.stack([t4[q] for q in packed_list4(t4.shape[0])])


def unpack_t4(t4p, o):
    """Full tensor from the stored blocks: block (p,q,r,s) is the stored block
    of the sorted indices with its virtual axes permuted the same way."""
    v = t4p.shape[1]
    full = np.empty((o,) * 4 + (v,) * 4)
    index = {q: n for n, q in enumerate(packed_list4(o))}
    for occ in itertools.product(range(o), repeat=4):
        order = sorted(range(4), key=lambda s: occ[s])
        blk = t4p[index[tuple(occ[s] for s in order)]]
        full[occ] = blk.transpose([order.index(s) for s in range(4)])
    return full
