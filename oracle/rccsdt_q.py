"""Perturbative quadruples correction E_(Q) of spin-restricted CCSDT(Q), FP64,
on full spin-free tensors (test oracle only).

Follows the paper's Appendix "(Q) energy correction" (Eq. ener-pt-q with the
residual Eq. resi-pt-q): from converged (or any) T2 and T3 and the bare
integrals,

  X_ijkl^abcd = 1/2 sum_e v^{ab}_{ej} t_ikl^ecd - 1/2 sum_m v^{am}_{ij} t_mkl^bcd
  V_ijkl^abcd = 1/4 v^{ab}_{ij} t_kl^cd
  Wbar_ejk^abc = P_(jb)(kc) [ 1/2 sum_f v^{ab}_{ef} t_jk^fc ]
  Wbar_ijk^abm = P_(ia)(jb) [ sum_e v^{ma}_{ei} t_jk^be + sum_e v^{ma}_{ke} t_ji^be
                              - 1/2 sum_n v^{mn}_{ki} t_nj^ab ]
  Y_ijkl^abcd = 1/2 sum_e Wbar_ejk^abc t_il^ed - 1/2 sum_m Wbar_ijk^abm t_ml^cd
  r = P_(ia)(jb)(kc)(ld) (X + Y),   z = P_(ia)(jb)(kc)(ld) (X + V)
  t4 = r / eps_ijkl^abcd   (eps = sum eps_occ - sum eps_vir, eps_p = f_pp)
  E_(Q) = 1/24 sum_ijklabcd z_ijkl^abcd tchk_ijkl^abcd

with P the unnormalised sum over simultaneous permutations of the listed
columns and the fully spin-summed quadruples amplitude (Eq. quadruples-spin-sum
and the (Q) appendix)

  u1 = (2 - P_a^b - P_a^c - P_a^d) t4
  u2 = (2 - P_b^c - P_b^d) u1
  tchk = 2 (2 - P_c^d) u2

where P_x^y exchanges two virtual labels with the occupied labels fixed.
Canonical orbitals are assumed (the denominators use the diagonal of f only,
as the paper's non-iterative amplitudes do).  T1 does not enter.

Array conventions as in oracle.rccsdt: V[p,q,r,s] = v^{pq}_{rs} (bare),
t2[i,j,a,b], t3[i,j,k,a,b,c], full tensors t4[i,j,k,l,a,b,c,d] (o^4 v^4
elements: small systems only).
"""

from __future__ import annotations

import itertools

import numpy as np

PERMS4 = list(itertools.permutations(range(4)))


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def perm_sym4(X: np.ndarray) -> np.ndarray:
    """P_(ia)(jb)(kc)(ld) X: sum over the 24 simultaneous permutations of the
    four (occupied, virtual) columns of X[i,j,k,l,a,b,c,d]."""
    out = np.zeros_like(X)
    for p in PERMS4:
        out += X.transpose(*p, *(4 + q for q in p))
    return out


def wbar_vvvo(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """Wbar_ejk^abc as W[e,j,k,a,b,c] (Eq. q_w_vvv_voo)."""
    Vs = slice(o, None)
    vvvv = V[Vs, Vs, Vs, Vs]                       # v^{ab}_{ef} = vvvv[a,b,e,f]
    half = 0.5 * _es("abef,jkfc->ejkabc", vvvv, t2)
    return half + half.transpose(0, 2, 1, 3, 5, 4)  # + (j,b) <-> (k,c)


def wbar_vooo(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """Wbar_ijk^abm as W[i,j,k,a,b,m] (Eq. q_w_vvo_ooo)."""
    O, Vs = slice(0, o), slice(o, None)
    g = (_es("maei,jkbe->ijkabm", V[O, Vs, Vs, O], t2)
         + _es("make,jibe->ijkabm", V[O, Vs, O, Vs], t2)
         - 0.5 * _es("mnki,njab->ijkabm", V[O, O, O, O], t2))
    return g + g.transpose(1, 0, 2, 4, 3, 5)        # + (i,a) <-> (j,b)


def x_term(V: np.ndarray, t3: np.ndarray, o: int) -> np.ndarray:
    """X_ijkl^abcd (Eq. q_t3_terms) as X[i,j,k,l,a,b,c,d]."""
    O, Vs = slice(0, o), slice(o, None)
    return (0.5 * _es("abej,iklecd->ijklabcd", V[Vs, Vs, Vs, O], t3)
            - 0.5 * _es("amij,mklbcd->ijklabcd", V[Vs, O, O, O], t3))


def y_term(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """Y_ijkl^abcd as Y[i,j,k,l,a,b,c,d]."""
    return (0.5 * _es("ejkabc,iled->ijklabcd", wbar_vvvo(V, t2, o), t2)
            - 0.5 * _es("ijkabm,mlcd->ijklabcd", wbar_vooo(V, t2, o), t2))


def v_term(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """V_ijkl^abcd = 1/4 v^{ab}_{ij} t_kl^cd."""
    O, Vs = slice(0, o), slice(o, None)
    return 0.25 * _es("abij,klcd->ijklabcd", V[Vs, Vs, O, O], t2)


def denominators4(f: np.ndarray, o: int) -> np.ndarray:
    e = np.diag(f)
    eo, ev = e[:o], e[o:]
    occ = eo[:, None, None, None] + eo[None, :, None, None] + eo[None, None, :, None] + eo[None, None, None, :]
    vir = ev[:, None, None, None] + ev[None, :, None, None] + ev[None, None, :, None] + ev[None, None, None, :]
    return occ[:, :, :, :, None, None, None, None] - vir[None, None, None, None]


def quadruples(f, V, t2, t3, o):
    """(t4, z): the non-iterative quadruples amplitudes and the energy weights."""
    X = x_term(V, t3, o)
    t4 = perm_sym4(X + y_term(V, t2, o)) / denominators4(f, o)
    z = perm_sym4(X + v_term(V, t2, o))
    return t4, z


def spin_sum4(t4: np.ndarray) -> np.ndarray:
    """Fully spin-summed quadruples amplitude from the spin-free one (virtual
    label exchanges at fixed occupied labels, applied in the order listed)."""
    def swap(x, p, q):
        ax = list(range(8))
        ax[4 + p], ax[4 + q] = ax[4 + q], ax[4 + p]
        return x.transpose(ax)
    u1 = 2.0 * t4 - swap(t4, 0, 1) - swap(t4, 0, 2) - swap(t4, 0, 3)
    u2 = 2.0 * u1 - swap(u1, 1, 2) - swap(u1, 1, 3)
    return 2.0 * (2.0 * u2 - swap(u2, 2, 3))


def energy_q(f, V, t2, t3, o) -> float:
    """E_(Q) = 1/24 sum z tchk."""
    t4, z = quadruples(f, V, t2, t3, o)
    return float(_es("ijklabcd,ijklabcd->", z, spin_sum4(t4)) / 24.0)


# ---------------------------------------------------------------------------
# One occupied tuple at a time (sizes where the o^4 v^4 tensors do not fit)
# ---------------------------------------------------------------------------

def _blocks_for(V, t2, t3, o, q):
    """X, Y and V blocks [a][b][c][d] of the ordered occupied tuple q, from
    the same expressions as x_term, y_term and v_term with the occupied
    indices fixed (t3 full [i][j][k][a][b][c])."""
    q0, q1, q2, q3 = q
    O, Vs = slice(0, o), slice(o, None)
    X = (0.5 * np.tensordot(V[Vs, Vs, Vs, q1], t3[q0, q2, q3], axes=([2], [0]))
         - 0.5 * np.tensordot(V[Vs, O, q0, q1], t3[:, q2, q3], axes=([1], [0])))
    vvvv = V[Vs, Vs, Vs, Vs]
    # Wbar_{e q1 q2}^{abc} = 1/2 sum_f v^{ab}_{ef} t_{q1 q2}^{fc} + 1/2 sum_f v^{ac}_{ef} t_{q2 q1}^{fb}, as [e][a][b][c]
    w1 = 0.5 * np.tensordot(vvvv, t2[q1, q2], axes=([3], [0]))            # [a][b][e][c]
    w2 = 0.5 * np.tensordot(vvvv, t2[q2, q1], axes=([3], [0]))            # [a][c][e][b]
    Wv = w1.transpose(2, 0, 1, 3) + w2.transpose(2, 0, 3, 1)
    Y = 0.5 * np.tensordot(Wv, t2[q0, q3], axes=([0], [0]))               # [a][b][c][d]

    def g(i, j, k):  # the bracket of Wbar_ijk^abm as [a][b][m]
        return (np.einsum("mae,be->abm", V[O, Vs, Vs, i], t2[j, k])
                + np.einsum("mae,be->abm", V[O, Vs, k, Vs], t2[j, i])
                - 0.5 * np.einsum("mn,nab->abm", V[O, O, k, i], t2[:, j]))

    Wo = g(q0, q1, q2) + g(q1, q0, q2).transpose(1, 0, 2)
    Y -= 0.5 * np.tensordot(Wo, t2[:, q3], axes=([2], [0]))
    Vb = 0.25 * np.multiply.outer(V[Vs, Vs, q0, q1], t2[q2, q3])
    return X, Y, Vb


def spin_sum_block(u):
    """spin_sum4 on one [a][b][c][d] block (the occupied labels fixed)."""
    def swap(x, p, q):
        ax = [0, 1, 2, 3]
        ax[p], ax[q] = ax[q], ax[p]
        return x.transpose(ax)
    u1 = 2.0 * u - swap(u, 0, 1) - swap(u, 0, 2) - swap(u, 0, 3)
    u2 = 2.0 * u1 - swap(u1, 1, 2) - swap(u1, 1, 3)
    return 2.0 * (2.0 * u2 - swap(u2, 2, 3))


def task_energy(f, V, t2, t3, o, task):
    """Contribution of the occupied tuple task = (i, j, k, l), i <= j <= k <= l,
    to E_(Q): sum over its distinct orderings q of sum_abcd (X + V)_q tchk_q,
    with tchk_q the fully spin-summed t4 block at q.  t4 at the tuple itself
    is the 24-permutation sum of (X + Y) blocks at the permuted tuples over
    the denominator; at another ordering q = the tuple permuted by p, tchk_q
    is tchk at the tuple with its virtual axes permuted the same way (the
    column symmetry of the spin-summed amplitudes)."""
    o_ = tuple(task)
    e = np.diag(f)
    eps_o = sum(e[x] for x in o_)
    ev = e[o:]
    den = eps_o - (ev[:, None, None, None] + ev[None, :, None, None] + ev[None, None, :, None]
                   + ev[None, None, None, :])
    cache = {}

    def blocks(q):
        if q not in cache:
            cache[q] = _blocks_for(V, t2, t3, o, q)
        return cache[q]

    r = 0.0
    for p in PERMS4:
        # full-tensor convention of perm_sym4: out[o][w] += G[o'][w'] with o'_{p[k]} = o_k
        qq = [0] * 4
        for k in range(4):
            qq[p[k]] = o_[k]
        X, Y, _ = blocks(tuple(qq))
        r = r + (X + Y).transpose(p)
    U = spin_sum_block(r / den)
    total = 0.0
    seen = set()
    for p in PERMS4:
        qq = [0] * 4
        for k in range(4):
            qq[p[k]] = o_[k]
        q = tuple(qq)
        if q in seen:
            continue
        seen.add(q)
        X, _, Vb = blocks(q)
        # tchk_q[w'] with w'_{p[k]} = w_k equals U[w]: U transposed by the inverse of p
        inv = [0] * 4
        for k in range(4):
            inv[p[k]] = k
        total += float(np.sum((X + Vb) * U.transpose(inv)))
    return total


# ---------------------------------------------------------------------------
# Alternative intermediates and the virtual-tuple summation order
# (Sec. "ABC-based algorithm", Eqs. q_w_alter and ener-pt-q-abc)
# ---------------------------------------------------------------------------

def wbar_vvvo_alt(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """The alternative Wbar_ejk^abc as W[e,j,k,a,b,c]:
    P_(jb)(kc) [ -sum_m v^{mb}_{ej} t_mk^ac - sum_m v^{ma}_{je} t_mk^bc
                 + 1/2 sum_f v^{ab}_{ef} t_jk^fc ]."""
    O, Vs = slice(0, o), slice(o, None)
    g = (-_es("mbej,mkac->ejkabc", V[O, Vs, Vs, O], t2)
         - _es("maje,mkbc->ejkabc", V[O, Vs, O, Vs], t2)
         + 0.5 * _es("abef,jkfc->ejkabc", V[Vs, Vs, Vs, Vs], t2))
    return g + g.transpose(0, 2, 1, 3, 5, 4)        # + (j,b) <-> (k,c)


def wbar_vooo_alt(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """The alternative Wbar_ijk^abm as W[i,j,k,a,b,m]:
    P_(ia)(jb) [ -1/2 sum_n v^{mn}_{ki} t_nj^ab ]."""
    O = slice(0, o)
    g = -0.5 * _es("mnki,njab->ijkabm", V[O, O, O, O], t2)
    return g + g.transpose(1, 0, 2, 4, 3, 5)        # + (i,a) <-> (j,b)


def y_term_alt(V: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """Y_ijkl^abcd built from the alternative intermediates (differs from
    y_term element by element; its 24-permutation sum is the same)."""
    return (0.5 * _es("ejkabc,iled->ijklabcd", wbar_vvvo_alt(V, t2, o), t2)
            - 0.5 * _es("ijkabm,mlcd->ijklabcd", wbar_vooo_alt(V, t2, o), t2))


def energy_q_by_virtual_tuples(f, V, t2, t3, o):
    """E_(Q) summed in the virtual-tuple order of Eq. ener-pt-q-abc:
    1/24 sum over a <= b <= c <= d of f_abcd sum_ijkl z tchk, f_abcd the
    number of distinct orderings of (a,b,c,d) (the summand is invariant under
    simultaneous permutations of the virtual labels of z and tchk with the
    occupied ones); returns (total, {virtual tuple: contribution})."""
    t4, z = quadruples(f, V, t2, t3, o)
    w = z * spin_sum4(t4)  # [i,j,k,l,a,b,c,d]
    per_abcd = w.sum(axis=(0, 1, 2, 3))
    v = per_abcd.shape[0]
    parts = {}
    for a in range(v):
        for b in range(a, v):
            for c in range(b, v):
                for d in range(c, v):
                    n = len(set(itertools.permutations((a, b, c, d))))
                    parts[(a, b, c, d)] = n * float(per_abcd[a, b, c, d]) / 24.0
    return sum(parts.values()), parts


def _blocks_for_virtual(V, t2, t3, o, q):
    """X, Y and V as o^4 arrays [i][j][k][l] for the ordered virtual tuple q
    (indices 0..v-1), from the same expressions as x_term, y_term_alt and
    v_term with the virtual indices fixed; Y uses the alternative
    intermediates of Eq. q_w_alter."""
    a, b, c, d = (o + x for x in q)
    O, Vs = slice(0, o), slice(o, None)
    qa, qb, qc, qd = q
    # X = 1/2 sum_e v^{ab}_{ej} t_ikl^{ecd} - 1/2 sum_m v^{am}_{ij} t_mkl^{bcd}
    X = (0.5 * _es("ej,ikle->ijkl", V[a, b, Vs, O], t3[:, :, :, :, qc, qd])
         - 0.5 * _es("mij,mkl->ijkl", V[a, O, O, O], t3[:, :, :, qb, qc, qd]))
    # alternative Wbar_ejk^{abc} for this (a,b,c) as [e][j][k]
    def gv(x, y, z):  # bracket of Eq. q_w_alter (vvv) for virtual labels (x, y, z) as [e][j][k]
        return (-_es("mej,mk->ejk", V[O, o + y, Vs, O], t2[:, :, x, z])
                - _es("mje,mk->ejk", V[O, o + x, O, Vs], t2[:, :, y, z])
                + 0.5 * _es("ef,jkf->ejk", V[o + x, o + y, Vs, Vs], t2[:, :, :, z]))
    Wv = gv(qa, qb, qc) + gv(qa, qc, qb).transpose(0, 2, 1)
    # alternative Wbar_ijk^{abm} for this (a,b) as [i][j][k][m]
    def gvo(x, y):
        return -0.5 * _es("mnki,nj->ijkm", V[O, O, O, O], t2[:, :, x, y])
    Wo = gvo(qa, qb) + gvo(qb, qa).transpose(1, 0, 2, 3)
    Y = (0.5 * _es("ejk,ile->ijkl", Wv, t2[:, :, :, qd])
         - 0.5 * _es("ijkm,ml->ijkl", Wo, t2[:, :, qc, qd]))
    Vb = 0.25 * np.multiply.outer(V[a, b, O, O], t2[:, :, qc, qd])
    return X, Y, Vb


def spin_sum_occ_block(u):
    """The spin summation of the virtual labels, acting on an o^4 array of a
    fixed virtual tuple: exchanging two virtual labels at fixed occupied ones
    equals exchanging the two occupied labels at fixed virtual ones (column
    symmetry), so the same operator applies to the occupied axes."""
    return spin_sum_block(u)


def virtual_task_energy(f, V, t2, t3, o, task):
    """Contribution of the virtual tuple task = (a, b, c, d), a <= b <= c <= d
    (indices 0..v-1), to E_(Q) in the order of Eq. ener-pt-q-abc: the mirror
    of task_energy with the roles of the occupied and virtual labels swapped
    (o^4 arrays per ordering of the virtual labels)."""
    t_ = tuple(task)
    e = np.diag(f)
    eps_v = sum(e[o + x] for x in t_)
    eo = e[:o]
    den = (eo[:, None, None, None] + eo[None, :, None, None] + eo[None, None, :, None]
           + eo[None, None, None, :]) - eps_v
    cache = {}

    def blocks(q):
        if q not in cache:
            cache[q] = _blocks_for_virtual(V, t2, t3, o, q)
        return cache[q]

    r = 0.0
    for p in PERMS4:
        qq = [0] * 4
        for k in range(4):
            qq[p[k]] = t_[k]
        X, Y, _ = blocks(tuple(qq))
        r = r + (X + Y).transpose(p)
    U = spin_sum_occ_block(r / den)
    total = 0.0
    seen = set()
    for p in PERMS4:
        qq = [0] * 4
        for k in range(4):
            qq[p[k]] = t_[k]
        q = tuple(qq)
        if q in seen:
            continue
        seen.add(q)
        X, _, Vb = blocks(q)
        inv = [0] * 4
        for k in range(4):
            inv[p[k]] = k
        total += float(np.sum((X + Vb) * U.transpose(inv)))
    return total
