"""Block-level FP64 oracle for large systems (test oracle only).

Test infrastructure: only tests, the smoke check and the CPU baseline of the
benchmark use this module; the HIP library never does.

At o=20, v=180 the full T3 tensor (o^3 v^3 doubles, 373 GB) does not fit in
host memory, so the plain full-tensor oracle of ``rccsdt`` cannot run.  This
module evaluates one output block R3[i,j,k,:,:,:] of the particle-particle
ladder term by its definition, for sampled blocks:

  R3_pp[ijk][abc] = P_{(ia)(jb)(kc)} 1/2 sum_de W^{ab}_{de} t_{ijk}^{dec}
  W^{ab}_{de}     = v~^{ab}_{de} + sum_lm v~^{lm}_{de} t_lm^ab

(Eq. resi-rccsdt and the W^{ab}_{de} intermediate of the RCCSDT appendix),
with the paired-index permutation operator written out as its six terms
(Eq. rcc-perm-op), each off-triangle T3 block rebuilt from the stored block
by the column symmetry (Eq. rccsdt-amps-symm), followed by the R3
post-processing of Sec. "Removing redundancies in RCC amplitudes".
The dressed integrals come from the T1-dressed density-fitting factors
(Appendix A, "T1-dressed formalism").  No compact rewriting is used: all six
permutations are contracted, so a block costs 6 v^5 multiply-adds.
"""

from __future__ import annotations

import itertools

import numpy as np

PERMS3 = list(itertools.permutations(range(3)))


def dressed_factors(B: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """B~^P = x B^P y^T with x = 1 - t1, y = 1 + t1^T, [t1]_{a,i} = t_i^a."""
    o, v = t1.shape
    n = o + v
    tm = np.zeros((n, n))
    tm[o:, :o] = t1.T
    x = np.eye(n) - tm
    y = np.eye(n) + tm.T
    return np.einsum("pt,Ptu,ru->Ppr", x, B, y, optimize=True)


def w_vvvv(Bt: np.ndarray, t2: np.ndarray, o: int) -> np.ndarray:
    """W^{ab}_{de} = v~^{ab}_{de} + sum_lm v~^{lm}_{de} t_lm^ab as W[a,b,d,e],
    one row a at a time.  v~^{pq}_{rs} = sum_P B~^P_{pr} B~^P_{qs}; the sums
    over P and over (l,m) are matrix products (a library primitive)."""
    naux, n, _ = Bt.shape
    v = n - o
    Bvv = np.ascontiguousarray(Bt[:, o:, o:])  # [P][a][d]
    Xbe = Bvv.reshape(naux, v * v)  # [P][(b,e)]
    Y = np.ascontiguousarray(Bt[:, :o, o:]).reshape(naux, o * v)  # [P][(l,d)]
    voovv = np.ascontiguousarray((Y.T @ Y).reshape(o, v, o, v).transpose(0, 2, 1, 3)).reshape(o * o, v * v)
    BvvT = np.ascontiguousarray(Bvv.transpose(1, 2, 0))  # [a][d][P]
    t2T = np.ascontiguousarray(t2.reshape(o * o, v, v).transpose(1, 2, 0))  # [a][b][(l,m)]
    W = np.empty((v, v, v, v))
    for a in range(v):
        # v~^{ab}_{de} = sum_P B~_{ad} B~_{be}: rows d, columns (b,e)
        row = (BvvT[a] @ Xbe).reshape(v, v, v).transpose(1, 0, 2)  # [b][d][e]
        W[a] = row + (t2T[a] @ voovv).reshape(v, v, v)
    return W


def unpack_block(stored: np.ndarray, occ: tuple[int, int, int]) -> np.ndarray:
    """t_{pqr}^{xyz} for occ = (p,q,r) from the stored block of sort(p,q,r):
    the column symmetry carries the virtual axes with the occupied ones."""
    order = sorted(range(3), key=lambda s: occ[s])
    inv = [order.index(s) for s in range(3)]
    return stored.transpose(inv)


def pp_block(W: np.ndarray, stored: np.ndarray, ijk: tuple[int, int, int]) -> np.ndarray:
    """Raw (not post-processed) PP contribution to the packed block (i,j,k):
    sum over the six simultaneous column permutations of
    1/2 sum_de W^{xy}_{de} t_{sigma(ijk)}^{dez}."""
    v = stored.shape[0]
    out = np.zeros((v, v, v))
    Wm = W.reshape(v * v, v * v)
    for p in PERMS3:
        occ = tuple(ijk[s] for s in p)
        t = unpack_block(stored, occ)  # t_{occ}^{d e z}
        y = 0.5 * (Wm @ t.reshape(v * v, v)).reshape(v, v, v)  # y[x,y,z]
        # this permutation contributes y at (x,y,z) = (a_p0, a_p1, a_p2)
        inv = [p.index(s) for s in range(3)]
        out += y.transpose(inv)
    return out


def postprocess_block(r: np.ndarray, ijk: tuple[int, int, int]) -> np.ndarray:
    """Symmetrize (i=j<k over the first two virtual axes, i<j=k over the last
    two, averaged), zero i=j=k blocks, subtract the mean over the six virtual
    permutations."""
    i, j, k = ijk
    if i == j == k:
        return np.zeros_like(r)
    if i == j:
        r = 0.5 * (r + r.transpose(1, 0, 2))
    elif j == k:
        r = 0.5 * (r + r.transpose(0, 2, 1))
    m = sum(r.transpose(p) for p in PERMS3) / 6.0
    return r - m


def _sum_perms(term_of_occ, ijk):
    """sum over the six simultaneous column permutations sigma of
    X_{sigma(ijk)}^{sigma(abc)}, where term_of_occ(occ) returns X_{occ}^{xyz}
    as an array [x][y][z] (Eq. rcc-perm-op written out)."""
    out = None
    for p in PERMS3:
        occ = tuple(ijk[s] for s in p)
        y = term_of_occ(occ)
        inv = [p.index(s) for s in range(3)]
        out = y.transpose(inv) if out is None else out + y.transpose(inv)
    return out


def f1_block(Fvv: np.ndarray, stored: np.ndarray, ijk) -> np.ndarray:
    """Raw F^a_d part of the Fock term of R3 for packed block (i,j,k):
    P[1/2 sum_d F^a_d t_{ijk}^{dbc}] (Eq. resi-rccsdt), Fvv[a][d]."""
    return _sum_perms(lambda occ: 0.5 * np.einsum("xd,dyz->xyz", Fvv, unpack_block(stored, occ)), ijk)


def d1_block(Wvvvo: np.ndarray, t2: np.ndarray, ijk) -> np.ndarray:
    """Raw T2 driver P[sum_d W^{ab}_{dj} t_{ik}^{dc}] for packed block (i,j,k);
    Wvvvo[a][b][d][j], t2[i][k][d][c] (Eq. resi-rccsdt)."""
    return _sum_perms(lambda occ: np.einsum("xyd,dz->xyz", Wvvvo[:, :, :, occ[1]], t2[occ[0], occ[2]]), ijk)


def d2_block(Wvooo: np.ndarray, t2: np.ndarray, ijk) -> np.ndarray:
    """Raw T2 driver P[-sum_l W^{al}_{ij} t_{lk}^{bc}] for packed block (i,j,k);
    Wvooo[a][l][i][j], t2[l][k][b][c] (Eq. resi-rccsdt)."""
    return _sum_perms(lambda occ: -np.einsum("xl,lyz->xyz", Wvooo[:, :, occ[0], occ[1]], t2[:, occ[2]]), ijk)


def local_terms_block(W, Fvv, Wvvvo, Wvooo, t2, stored, ijk, terms=("PP", "F1", "D1", "D2")):
    """Post-processed sum of the R3 terms that need only this block of T3
    (particle-particle ladder, F_vv term, both T2 drivers)."""
    v = stored.shape[0]
    r = np.zeros((v, v, v))
    if "PP" in terms:
        r += pp_block(W, stored, ijk)
    if "F1" in terms:
        r += f1_block(Fvv, stored, ijk)
    if "D1" in terms:
        r += d1_block(Wvvvo, t2, ijk)
    if "D2" in terms:
        r += d2_block(Wvooo, t2, ijk)
    return postprocess_block(r, ijk)


def occ_virt_gram(Bt: np.ndarray, o: int) -> np.ndarray:
    """G[l][d][m][e] = v~^{lm}_{de} = sum_P B~^P_{ld} B~^P_{me} (a matrix product
    over the fitting index)."""
    naux, n, _ = Bt.shape
    v = n - o
    Y = np.ascontiguousarray(Bt[:, :o, o:]).reshape(naux, o * v)
    return (Y.T @ Y).reshape(o, v, o, v)


def local_terms_elements(Bt, t2, Fvv, Wvvvo, Wvooo, stored, ijk, abcs, G):
    """Post-processed values R3[ijk][a][b][c] of the block-local terms (ladder,
    F_vv term, both T2 drivers) for the listed (a,b,c), by definition: the raw
    value of every member of the (a,b,c) orbit as the sum over the six
    simultaneous column permutations, each W^{xy}_{de} row built on demand
    from the dressed factors, then the post-processing of the orbit.  For
    sizes where neither W nor a whole block's ladder fits a check."""
    o = t2.shape[0]
    v = stored.shape[0]
    rows = {}

    def wrow(x, y):
        if (x, y) not in rows:
            bx = Bt[:, o + x, o:]
            by = Bt[:, o + y, o:]
            rows[(x, y)] = bx.T @ by + np.einsum("lm,ldme->de", t2[:, :, x, y], G)
        return rows[(x, y)]

    views = {}

    def tview(occ):
        if occ not in views:
            views[occ] = unpack_block(stored, occ)
        return views[occ]

    def raw(abc):
        total = 0.0
        for p in PERMS3:
            p_, q_, r_ = (ijk[s] for s in p)
            x, y, z = (abc[s] for s in p)
            t = tview((p_, q_, r_))
            total += 0.5 * float(np.sum(wrow(x, y) * t[:, :, z]))                 # ladder
            total += 0.5 * float(Fvv[x] @ t[:, y, z])                             # F_vv
            total += float(Wvvvo[x, y, :, q_] @ t2[p_, r_, :, z])                 # W^{xy}_{dq} t_{pr}^{dz}
            total -= float(Wvooo[x, :, p_, q_] @ t2[:, r_, y, z])                 # W^{xl}_{pq} t_{lr}^{yz}
        return total

    i, j, k = ijk
    out = []
    for abc in abcs:
        if i == j == k:
            out.append(0.0)
            continue
        orbit = {}
        for p in PERMS3:
            m = tuple(abc[s] for s in p)
            if m not in orbit:
                orbit[m] = raw(m)

        def sym(m):
            if i == j:
                return 0.5 * (orbit[m] + orbit[(m[1], m[0], m[2])])
            if j == k:
                return 0.5 * (orbit[m] + orbit[(m[0], m[2], m[1])])
            return orbit[m]

        mean = sum(sym(tuple(abc[s] for s in p)) for p in PERMS3) / 6.0
        out.append(sym(tuple(abc)) - mean)
    return np.array(out)
