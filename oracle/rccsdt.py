"""Spin-restricted CCSDT on full spin-free tensors, FP64 (test oracle only).

Follows the paper's Appendix A: the T1-dressed Hamiltonian, the RCCSD
singles/doubles residuals and intermediates, the RCCSDT additions (T3 terms in
R1/R2, the intermediates W^{ab}_{dj}, W^{al}_{ij}, Wbar, W^{ab}_{de}) and the
triples residual (Eq. resi-rccsdt) with the unnormalised paired-index
permutation operator (Eq. rcc-perm-op).  The compact algorithm of the paper is
an exact rewriting of these equations restricted to i <= j <= k, so this full
tensor form is the plain definition the GPU path must reproduce.

Array conventions (all row-major numpy, FP64):
  V[p,q,r,s] = v^{pq}_{rs} = <pq|rs> = (pr|qs)   (physicists' notation)
  fd[p,q]    = f^p_q (row p, column q)
  t1[i,a], t2[i,j,a,b], t3[i,j,k,a,b,c]
A check mark on the first column ("spin summation") is a fixed linear
combination of index orders; see vchk, chk2, chk3_1 and chk3_12 below.
"""

from __future__ import annotations

import itertools

import numpy as np

PERMS3 = list(itertools.permutations(range(3)))


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


# ----------------------------------------------------------------------------
# Integrals and T1 dressing (Appendix A, "T1-dressed formalism")
# ----------------------------------------------------------------------------

def eri_phys_from_B(B: np.ndarray) -> np.ndarray:
    """v^{pq}_{rs} = (pr|qs) with (pq|rs) = sum_P B[P,p,q] B[P,r,s]."""
    chem = _es("Ppq,Prs->pqrs", B, B)
    return np.ascontiguousarray(chem.transpose(0, 2, 1, 3))


def t1_matrix(t1: np.ndarray, n: int) -> np.ndarray:
    """Embed singles into the n x n orbital space: [t1]_{a,i} = t_i^a."""
    o, v = t1.shape
    m = np.zeros((n, n))
    m[o:, :o] = t1.T
    return m


def dress(f: np.ndarray, V: np.ndarray, t1: np.ndarray):
    """T1-dressed integrals.  x = 1 - t1, y = 1 + t1^T;
    vt^{pq}_{rs} = sum x_pt x_qu v^{tu}_{vw} y_rv y_sw;
    ft = x [f + G] y^T with G_rs = sum_ia (2 v^{ri}_{sa} - v^{ri}_{as}) t_i^a."""
    o, v = t1.shape
    n = o + v
    tm = t1_matrix(t1, n)
    x = np.eye(n) - tm
    y = np.eye(n) + tm.T
    Vt = _es("pt,qu,tuvw,rv,sw->pqrs", x, x, V, y, y)
    G = 2.0 * _es("risa,ia->rs", V[:, :o, :, o:], t1) - _es("rias,ia->rs", V[:, :o, o:, :], t1)
    ft = x @ (f + G) @ y.T
    return ft, Vt


# ----------------------------------------------------------------------------
# Spin-summation helpers (check marks on the first column)
# ----------------------------------------------------------------------------

def vchk(V: np.ndarray) -> np.ndarray:
    """v^{p'q}_{r's} = 2 v^{pq}_{rs} - v^{pq}_{sr} (check on column 1)."""
    return 2.0 * V - V.transpose(0, 1, 3, 2)


def chk2(t2: np.ndarray) -> np.ndarray:
    """t_{i'j}^{a'b} = 2 t_ij^ab - t_ij^ba."""
    return 2.0 * t2 - t2.transpose(0, 1, 3, 2)


def chk3_1(t3: np.ndarray) -> np.ndarray:
    """Single check on column 1: (2 - P_a^b - P_a^c) t^{abc}
    = 2 X^{abc} - X^{bac} - X^{cba}, occupied labels fixed."""
    return 2.0 * t3 - t3.transpose(0, 1, 2, 4, 3, 5) - t3.transpose(0, 1, 2, 5, 4, 3)


def chk3_12(t3: np.ndarray) -> np.ndarray:
    """Double check on columns 1,2: (2 - P_b^c)(2 - P_a^b - P_a^c) t^{abc}
    (Eq. triples-spin-sum), acting on virtual positions with occupied fixed."""
    s1 = chk3_1(t3)
    return 2.0 * s1 - s1.transpose(0, 1, 2, 3, 5, 4)


def perm_sym3(X: np.ndarray) -> np.ndarray:
    """Unnormalised P_{(ia)(jb)(kc)}: sum over the 6 simultaneous column
    permutations of an (o,o,o,v,v,v) tensor."""
    out = np.zeros_like(X)
    for p in PERMS3:
        out += X.transpose(p[0], p[1], p[2], 3 + p[0], 3 + p[1], 3 + p[2])
    return out


# ----------------------------------------------------------------------------
# Intermediates
# ----------------------------------------------------------------------------

def slices(o, n):
    return slice(0, o), slice(o, n)


def ccsd_intermediates(ft, Vt, t2, o):
    """RCCSD intermediates F^b_c, F^k_j, W^{kl}_{ij}, W^{ka}_{ci}, W^{ka}_{ic}."""
    n = ft.shape[0]
    O, Vs = slices(o, n)
    Vc = vchk(Vt)
    tau = chk2(t2)
    Fvv = ft[Vs, Vs] - _es("kldc,kldb->bc", Vc[O, O, Vs, Vs], t2)
    Foo = ft[O, O] + _es("lkcd,ljcd->kj", Vc[O, O, Vs, Vs], t2)
    Woooo = Vt[O, O, O, O] + _es("klcd,ijcd->klij", Vt[O, O, Vs, Vs], t2)
    Wovvo = Vc[O, Vs, Vs, O] + 0.5 * _es("lkdc,lida->kaci", Vc[O, O, Vs, Vs], tau)
    Wovov = Vt[O, Vs, O, Vs] - 0.5 * _es("lkcd,ilda->kaic", Vt[O, O, Vs, Vs], t2)
    return dict(Fvv=Fvv, Foo=Foo, Woooo=Woooo, Wovvo=Wovvo, Wovov=Wovov)


def ccsdt_intermediates(ft, Vt, t2, t3, o, ims):
    """RCCSDT intermediates W^{ab}_{dj}, W^{al}_{ij}, Wbar^{la}_{di},
    Wbar^{la}_{id}, W^{ab}_{de}, including their T3 parts."""
    n = ft.shape[0]
    O, Vs = slices(o, n)
    Vc = vchk(Vt)
    tau = chk2(t2)
    s1 = chk3_1(t3) if t3 is not None else None
    fov = ft[O, Vs]
    Wvvvo = (Vt[Vs, Vs, Vs, O]
             + 0.5 * _es("laed,ljeb->abdj", Vc[O, Vs, Vs, Vs], tau)
             - 0.5 * _es("lade,jleb->abdj", Vt[O, Vs, Vs, Vs], t2)
             - _es("lbde,jlea->abdj", Vt[O, Vs, Vs, Vs], t2)
             + _es("lmdj,lmab->abdj", Vt[O, O, Vs, O], t2))
    Wvooo = (Vt[Vs, O, O, O]
             + _es("ld,ijad->alij", fov, t2)
             + 0.5 * _es("mldj,mida->alij", Vc[O, O, Vs, O], tau)
             - 0.5 * _es("mljd,imda->alij", Vt[O, O, O, Vs], t2)
             - _es("mlid,jmda->alij", Vt[O, O, O, Vs], t2)
             + _es("alde,ijde->alij", Vt[Vs, O, Vs, Vs], t2))
    if s1 is not None:
        Wvvvo = Wvvvo - _es("lmde,mjleba->abdj", Vt[O, O, Vs, Vs], s1)
        Wvooo = Wvooo + _es("lmde,mijead->alij", Vt[O, O, Vs, Vs], s1)
    Wbar_ovvo = ims["Wovvo"] + 0.5 * _es("mled,miea->ladi", Vc[O, O, Vs, Vs], tau)
    Wbar_ovov = ims["Wovov"] - 0.5 * _es("mlde,imea->laid", Vt[O, O, Vs, Vs], t2)
    Wvvvv = Vt[Vs, Vs, Vs, Vs] + _es("lmde,lmab->abde", Vt[O, O, Vs, Vs], t2)
    return dict(Wvvvo=Wvvvo, Wvooo=Wvooo, Wbar_ovvo=Wbar_ovvo, Wbar_ovov=Wbar_ovov, Wvvvv=Wvvvv)


# ----------------------------------------------------------------------------
# Residuals
# ----------------------------------------------------------------------------

R3_TERMS = ("D1", "D2", "F1", "F2", "RA", "RB", "RC", "HH", "PP")


_R3_TERM_EXPR = {
    "D1": lambda t2, t3, ims, ims3: _es("abdj,ikdc->ijkabc", ims3["Wvvvo"], t2),
    "D2": lambda t2, t3, ims, ims3: -_es("alij,lkbc->ijkabc", ims3["Wvooo"], t2),
    "F1": lambda t2, t3, ims, ims3: 0.5 * _es("ad,ijkdbc->ijkabc", ims["Fvv"], t3),
    "F2": lambda t2, t3, ims, ims3: -0.5 * _es("li,ljkabc->ijkabc", ims["Foo"], t3),
    "RA": lambda t2, t3, ims, ims3: 0.25 * _es("ladi,ljkdbc->ijkabc", ims3["Wbar_ovvo"], chk3_1(t3)),
    "RB": lambda t2, t3, ims, ims3: -0.5 * _es("laid,jlkdbc->ijkabc", ims3["Wbar_ovov"], t3),
    "RC": lambda t2, t3, ims, ims3: -_es("lbid,jlkdac->ijkabc", ims3["Wbar_ovov"], t3),
    "HH": lambda t2, t3, ims, ims3: 0.5 * _es("lmij,lmkabc->ijkabc", ims["Woooo"], t3),
    "PP": lambda t2, t3, ims, ims3: 0.5 * _es("abde,ijkdec->ijkabc", ims3["Wvvvv"], t3),
}


def r3_term(name, t2, t3, ims, ims3):
    """One of the nine terms inside P_{(ia)(jb)(kc)} of Eq. resi-rccsdt, as a
    full (o,o,o,v,v,v) tensor before the permutation operator."""
    return _R3_TERM_EXPR[name](t2, t3, ims, ims3)


def r3_terms(t2, t3, ims, ims3):
    """All nine terms (see r3_term), in the order D1 D2 F1 F2 RA RB RC HH PP."""
    return {name: r3_term(name, t2, t3, ims, ims3) for name in _R3_TERM_EXPR}


def residuals(f, V, t1, t2, t3, o, triples=True, terms=None, return_parts=False):
    """Raw residuals (R1, R2, R3) of RCCSDT (or RCCSD if ``triples`` is False).

    R3 is returned before post-processing.  ``terms`` optionally restricts R3 to
    a subset of R3_TERMS (each term is still passed through the permutation
    operator)."""
    n = f.shape[0]
    O, Vs = slices(o, n)
    v = n - o
    ft, Vt = dress(f, V, t1)
    ims = ccsd_intermediates(ft, Vt, t2, o)
    tau = chk2(t2)
    fov = ft[O, Vs]

    # Singles (Eq. ccsd_r1 and its RCCSDT T3 term)
    r1 = ft[Vs, O].T.copy()
    r1 += _es("kc,ikac->ia", fov, tau)
    r1 += _es("akcd,ikcd->ia", Vt[Vs, O, Vs, Vs], tau)
    r1 -= _es("klic,klac->ia", Vt[O, O, O, Vs], tau)

    # Doubles (Eq. ccsd_r2), before P_{(ia)(jb)}
    X2 = 0.5 * Vt[Vs, Vs, O, O].transpose(2, 3, 0, 1)
    X2 = X2 + _es("bc,ijac->ijab", ims["Fvv"], t2)
    X2 -= _es("kj,ikab->ijab", ims["Foo"], t2)
    X2 += 0.5 * _es("abcd,ijcd->ijab", Vt[Vs, Vs, Vs, Vs], t2)
    X2 += 0.5 * _es("klij,klab->ijab", ims["Woooo"], t2)
    X2 += 0.5 * _es("kaci,kjcb->ijab", ims["Wovvo"], tau)
    X2 -= 0.5 * _es("kaic,jkcb->ijab", ims["Wovov"], t2)
    X2 -= _es("kbic,jkca->ijab", ims["Wovov"], t2)

    r3 = None
    parts = None
    if triples:
        if t3 is None:
            t3 = np.zeros((o, o, o, v, v, v))
        s1 = chk3_1(t3)
        r1 += 0.5 * _es("jkbc,jkibca->ia", Vt[O, O, Vs, Vs], chk3_12(t3))
        X2 += 0.5 * _es("kc,kijcab->ijab", fov, s1)
        X2 += _es("bkcd,kijdac->ijab", Vt[Vs, O, Vs, Vs], s1)
        X2 -= _es("kljc,likcab->ijab", Vt[O, O, O, Vs], s1)
        ims3 = ccsdt_intermediates(ft, Vt, t2, t3, o, ims)
        use = R3_TERMS if terms is None else terms
        X3 = np.zeros((o, o, o, v, v, v))
        if return_parts:
            parts = r3_terms(t2, t3, ims, ims3)
            for name in use:
                X3 += parts[name]
        else:
            # one term at a time (same sum, same order; only one term tensor alive)
            for name in use:
                X3 += r3_term(name, t2, t3, ims, ims3)
        r3 = perm_sym3(X3)
    r2 = X2 + X2.transpose(1, 0, 3, 2)
    if return_parts:
        return r1, r2, r3, parts
    return r1, r2, r3


# ----------------------------------------------------------------------------
# R3 post-processing (Sec. "Removing redundancies in RCC amplitudes")
# ----------------------------------------------------------------------------

def symmetrize_r3(r3: np.ndarray) -> np.ndarray:
    """Average blocks with two equal occupied indices over the swap of the
    corresponding virtual indices: i=j<k over (a,b), i<j=k over (b,c).  On a
    full tensor produced by the permutation operator this only removes
    roundoff."""
    r = r3.copy()
    o = r.shape[0]
    for i in range(o):
        for k in range(i + 1, o):
            blk = r3[i, i, k]
            r[i, i, k] = 0.5 * (blk + blk.transpose(1, 0, 2))
            blk = r3[i, k, k]
            r[i, k, k] = 0.5 * (blk + blk.transpose(0, 2, 1))
    return r


def purify_r3(r3: np.ndarray) -> np.ndarray:
    """Zero the i=j=k blocks (three equal spatial holes cannot exist)."""
    r = r3.copy()
    for i in range(r.shape[0]):
        r[i, i, i] = 0.0
    return r


def orthogonalize_r3(r3: np.ndarray) -> np.ndarray:
    """R3 <- (1 - Pi_[3]) R3: subtract the mean over the six permutations of
    the virtual indices (null space of the spin-free triples overlap)."""
    m = np.zeros_like(r3)
    for p in PERMS3:
        m += r3.transpose(0, 1, 2, 3 + p[0], 3 + p[1], 3 + p[2])
    return r3 - m / 6.0


def postprocess_r3(r3: np.ndarray) -> np.ndarray:
    return orthogonalize_r3(purify_r3(symmetrize_r3(r3)))


# ----------------------------------------------------------------------------
# Energy, denominators, update, norms
# ----------------------------------------------------------------------------

def energy(f, V, t1, t2, o):
    """E = sum_ijab (2 v^{ij}_{ab} - v^{ij}_{ba}) (t_ij^ab + t_i^a t_j^b)
    + 2 sum_ia f^i_a t_i^a, with the bare (undressed) v and f."""
    n = f.shape[0]
    O, Vs = slices(o, n)
    Vc = vchk(V)[O, O, Vs, Vs]
    tau = t2 + _es("ia,jb->ijab", t1, t1)
    return float(_es("ijab,ijab->", Vc, tau) + 2.0 * _es("ia,ia->", f[O, Vs], t1))


def denominators(f, o):
    """Orbital-energy denominators eps_{i..}^{a..} = sum eps_occ - sum eps_vir,
    with eps_p = f_pp of the bare Fock matrix."""
    e = np.diag(f)
    eo, ev = e[:o], e[o:]
    d1 = eo[:, None] - ev[None, :]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    d3 = (eo[:, None, None, None, None, None] + eo[None, :, None, None, None, None] + eo[None, None, :, None, None, None]
          - ev[None, None, None, :, None, None] - ev[None, None, None, None, :, None] - ev[None, None, None, None, None, :])
    return d1, d2, d3


def mp2_guess(f, V, o):
    """T1 = 0, T2 = v^{ij}_{ab} / eps_ij^ab, T3 = 0."""
    n = f.shape[0]
    O, Vs = slices(o, n)
    d1, d2, d3 = denominators(f, o)
    t1 = np.zeros(d1.shape)
    t2 = V[O, O, Vs, Vs] / d2
    t3 = np.zeros(d3.shape)
    return t1, t2, t3


def residual_norm2(r1, r2, r3):
    """Squared full-tensor Frobenius norms of R1, R2, R3."""
    n3 = 0.0 if r3 is None else float(np.sum(r3 * r3))
    return float(np.sum(r1 * r1)), float(np.sum(r2 * r2)), n3


class DIIS:
    """Pulay DIIS on the concatenated (T1, T2, T3) vector.

    The error vector is e = T_jacobi - T_old, the extrapolated vectors are the
    Jacobi-updated ones, the inner product is the full-tensor Euclidean one,
    the space holds at most ``space`` vectors, extrapolation starts once
    ``start`` vectors are stored, and the bordered system is solved by LU with
    partial pivoting; a singular system drops the oldest vector and retries."""

    def __init__(self, space=8, start=2):
        self.space = space
        self.start = start
        self.vecs = []
        self.errs = []

    def update(self, vec_new, err):
        self.vecs.append(vec_new.copy())
        self.errs.append(err.copy())
        if len(self.vecs) > self.space:
            self.vecs.pop(0)
            self.errs.pop(0)
        if len(self.vecs) < self.start:
            return vec_new
        while True:
            m = len(self.vecs)
            Bm = np.empty((m + 1, m + 1))
            Bm[m, :] = -1.0
            Bm[:, m] = -1.0
            Bm[m, m] = 0.0
            for a in range(m):
                for b in range(a, m):
                    Bm[a, b] = Bm[b, a] = float(np.dot(self.errs[a], self.errs[b]))
            rhs = np.zeros(m + 1)
            rhs[m] = -1.0
            try:
                c = np.linalg.solve(Bm, rhs)
            except np.linalg.LinAlgError:
                c = None
            if c is None or not np.all(np.isfinite(c)):
                if m <= 1:
                    return vec_new
                self.vecs.pop(0)
                self.errs.pop(0)
                continue
            out = np.zeros_like(vec_new)
            for a in range(m):
                out += c[a] * self.vecs[a]
            return out


def pack_vec(t1, t2, t3):
    parts = [t1.ravel(), t2.ravel()]
    if t3 is not None:
        parts.append(t3.ravel())
    return np.concatenate(parts)


def unpack_vec(vec, o, v, triples=True):
    n1, n2 = o * v, o * o * v * v
    t1 = vec[:n1].reshape(o, v).copy()
    t2 = vec[n1:n1 + n2].reshape(o, o, v, v).copy()
    t3 = vec[n1 + n2:].reshape(o, o, o, v, v, v).copy() if triples else None
    return t1, t2, t3


def iterate(f, V, t1, t2, t3, o, triples=True, diis=None, diis_t3="full"):
    """One iteration: residuals, R3 post-processing, norms, Jacobi update
    t <- t + r / eps, optional DIIS, energy of the new amplitudes.

    diis_t3 selects the part of T3 in the DIIS vectors (Sec. "Distributed
    DIIS"): "full", "none" (T1/T2 only; T3 keeps its Jacobi step), or an int
    nv: only the components whose three virtual indices lie in the
    low-energy subspace (the first nv virtuals) enter the overlaps and are
    extrapolated; the rest of T3 keeps its Jacobi step.

    Returns (t1, t2, t3, energy, (|R1|^2, |R2|^2, |R3|^2))."""
    r1, r2, r3 = residuals(f, V, t1, t2, t3, o, triples=triples)
    if triples:
        r3 = postprocess_r3(r3)
    norms = residual_norm2(r1, r2, r3)
    d1, d2, d3 = denominators(f, o)
    n1 = t1 + r1 / d1
    n2 = t2 + r2 / d2
    n3 = t3 + r3 / d3 if triples else None
    if diis is not None:
        v = t1.shape[1]
        if not triples or diis_t3 == "none":
            sub = 0
        elif diis_t3 == "full":
            sub = v
        else:
            sub = int(diis_t3)
        part = (lambda x: x[:, :, :, :sub, :sub, :sub]) if sub else (lambda x: None)
        new = pack_vec(n1, n2, part(n3) if triples else None)
        old = pack_vec(t1, t2, part(t3) if triples else None)
        out = diis.update(new, new - old)
        n_12 = o * v + o * o * v * v
        n1 = out[:o * v].reshape(o, v).copy()
        n2 = out[o * v:n_12].reshape(o, o, v, v).copy()
        if sub:
            n3 = n3.copy()
            n3[:, :, :, :sub, :sub, :sub] = out[n_12:].reshape(o, o, o, sub, sub, sub)
    e = energy(f, V, n1, n2, o)
    return n1, n2, n3, e, norms


def solve(f, V, o, triples=True, max_iter=200, tol=1e-10, diis=True, t_init=None, verbose=False, diis_t3="full"):
    """Iterate from the MP2 guess until sqrt(sum of squared norms) < tol.
    Returns (energy, t1, t2, t3, iterations, converged)."""
    if t_init is None:
        t1, t2, t3 = mp2_guess(f, V, o)
    else:
        t1, t2, t3 = t_init
    if not triples:
        t3 = None
    d = DIIS() if diis else None
    e = energy(f, V, t1, t2, o)
    for it in range(1, max_iter + 1):
        t1, t2, t3, e, nrm = iterate(f, V, t1, t2, t3, o, triples=triples, diis=d, diis_t3=diis_t3)
        rn = np.sqrt(sum(nrm))
        if verbose:
            print(it, e, rn)
        if rn < tol:
            return e, t1, t2, t3, it, True
    return e, t1, t2, t3, max_iter, False


# ----------------------------------------------------------------------------
# Packed (i <= j <= k) storage, for comparison with packed outputs
# ----------------------------------------------------------------------------

def packed_list(o):
    """Occupied triples i <= j <= k in lexicographic order."""
    return [(i, j, k) for i in range(o) for j in range(i, o) for k in range(j, o)]


def pack_t3(t3: np.ndarray) -> np.ndarray:
    """Restrict a full column-symmetric tensor to its stored blocks."""
    o = t3.shape[0]
    return np.stack([t3[i, j, k] for (i, j, k) in packed_list(o)])


def unpack_t3(t3p: np.ndarray, o: int) -> np.ndarray:
    """Rebuild the full tensor from stored blocks with the column symmetry:
    block (p,q,r) is the stored block sort(p,q,r) with its virtual axes
    permuted the same way."""
    v = t3p.shape[1]
    full = np.empty((o, o, o, v, v, v))
    index = {t: n for n, t in enumerate(packed_list(o))}
    for p in range(o):
        for q in range(o):
            for r in range(o):
                occ = (p, q, r)
                order = sorted(range(3), key=lambda s: occ[s])
                blk = t3p[index[tuple(occ[s] for s in order)]]
                # stored block axes are (order[0], order[1], order[2]) positions
                inv = [order.index(s) for s in range(3)]
                full[p, q, r] = blk.transpose(inv)
    return full


def multiplicity(i, j, k):
    """Number of distinct orderings of (i,j,k): 6, 3 or 1."""
    if i == j == k:
        return 1
    if i == j or j == k:
        return 3
    return 6
