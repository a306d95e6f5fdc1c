"""Seeded synthetic inputs for the compact-triples CCSDT residual.

This module produces input data only: orbital energies, density-fitting
factors B^P_pq, Fock matrices and test amplitudes.  It contains none of the
method's arithmetic (no dressing, no residual terms, no projections), so both
the oracle and the HIP path may take their inputs from it.

Recipe for a closed-shell system with ``o`` occupied and ``v`` virtual spatial
orbitals (n = o + v), ``naux`` fitting functions and a seed::

    rng   = numpy.random.default_rng(seed)               # PCG64
    eps_o = sort(rng.uniform(-1.5, -0.5, o))
    eps_v = sort(rng.uniform(0.3, 3.0, v))
    B     = rng.normal(0.0, 0.05, (naux, n, n))
    B     = triu(B) + swapaxes(triu(B, 1), 1, 2)          # B[P] symmetric in (p, q)
    f     = diag(concat(eps_o, eps_v))

so that (pq|rs) = sum_P B[P,p,q] B[P,r,s].  The paper's workloads are
molecules; these synthetic systems stand in for them at the paper's
occupied/virtual ratios.

With sigma fixed at 0.05 the exchange-type integrals (ia|ia) ~ naux sigma^2
grow with naux (0.12 / 0.50 / 1.00 at naux = 48 / 200 / 400) and the larger
named systems have no coupled-cluster solution reachable from the MP2 guess.
``scaled_sigma(naux)`` = 0.05 sqrt(48 / naux) keeps every (pq|rs) at the
variance of the o=4, v=20 system; the "-scaled" variants of the named
workloads (``make_named``) use it where a converged energy is needed.  At
o=20, v=180 even the scaled integrals couple too strongly: the iteration from
MP2 grows the residual about tenfold per step.  The "-weak" variant divides
the scaled standard deviation by three (correlation energy about 1 % of the
scaled one's MP2 value); from MP2 its residual norm falls by a factor of
about 2.5 per iteration, so a converged energy exists at that size.
"""

from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "CONFIGS",
    "make_system",
    "make_named",
    "scaled_sigma",
    "variant_sigma",
    "batched_sizes",
    "random_fock",
    "random_amplitudes",
    "random_t3_packed",
    "packed_triples",
    "hashed_t3_slab",
    "hashed_uniform",
]

# Named workloads: (o, v, naux, seed).
CONFIGS = {
    "o4v20": (4, 20, 48, 1),
    "o10v90": (10, 90, 200, 2),
    "o20v180": (20, 180, 400, 3),
    "o50v400": (50, 400, 900, 5),
}


def scaled_sigma(naux: int) -> float:
    """Entry standard deviation giving (pq|rs) the variance of naux = 48, sigma = 0.05."""
    return 0.05 * float(np.sqrt(48.0 / naux))


def variant_sigma(variant: str, naux: int) -> float:
    """Entry standard deviation of a workload variant: "" (0.05), "scaled"
    (scaled_sigma) or "weak" (scaled_sigma / 3)."""
    if variant == "":
        return 0.05
    if variant == "scaled":
        return scaled_sigma(naux)
    if variant == "weak":
        return scaled_sigma(naux) / 3.0
    raise ValueError(f"unknown workload variant {variant!r}")


def make_named(name: str) -> dict:
    """A named workload ("o10v90"), or its variance-scaled ("o10v90-scaled")
    or weak-coupling ("o20v180-weak") variant."""
    base, _, variant = name.partition("-")
    o, v, naux, seed = CONFIGS[base]
    return make_system(o, v, naux, seed, sigma=variant_sigma(variant, naux))


def make_system(o: int, v: int, naux: int | None = None, seed: int = 0, sigma: float = 0.05) -> dict:
    """Closed-shell synthetic system: bare Fock ``f`` (n x n), factors ``B``
    (naux x n x n, symmetric in the last two axes), orbital energies ``eps``.
    ``sigma`` is the standard deviation of the entries of B (0.05 in every
    named workload; tiny brute-force tests raise it to get sizeable
    correlation)."""
    if o < 1 or v < 1:
        raise ValueError("need o >= 1 and v >= 1")
    n = o + v
    if naux is None:
        naux = 2 * n
    rng = np.random.default_rng(seed)
    eps_o = np.sort(rng.uniform(-1.5, -0.5, o))
    eps_v = np.sort(rng.uniform(0.3, 3.0, v))
    B = rng.normal(0.0, sigma, (naux, n, n))
    B = np.triu(B) + np.swapaxes(np.triu(B, 1), 1, 2)
    eps = np.concatenate([eps_o, eps_v])
    f = np.diag(eps)
    return {"o": o, "v": v, "naux": naux, "seed": seed, "f": f, "B": np.ascontiguousarray(B), "eps": eps}


def batched_sizes(nsys: int = 64, seed: int = 4) -> list[tuple[int, int, int, int]]:
    """Sizes of the batch of independent small systems: o uniform in [3, 8],
    v uniform in [20, 60], naux = 2(o+v); system s uses seed 4000 + s."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(nsys):
        o = int(rng.integers(3, 9))
        v = int(rng.integers(20, 61))
        out.append((o, v, 2 * (o + v), 4000 + s))
    return out


def random_fock(o: int, v: int, seed: int, offdiag: float = 0.05) -> np.ndarray:
    """Symmetric, non-diagonal Fock matrix (orbital energies on the diagonal
    from the standard recipe plus small symmetric off-diagonal noise)."""
    sysd = make_system(o, v, 2, seed)
    rng = np.random.default_rng(seed + 7919)
    n = o + v
    X = rng.normal(0.0, offdiag, (n, n))
    return sysd["f"] + 0.5 * (X + X.T) - np.diag(np.diag(X))


def _col_perms(rank: int):
    return list(itertools.permutations(range(rank)))


def random_amplitudes(o: int, v: int, seed: int, scale1: float = 0.02, scale2: float = 0.02,
                      scale3: float = 0.01, triples: bool = True):
    """Random test amplitudes with the required column-permutation symmetry.

    t1[i,a]; t2[i,j,a,b] with t2[i,j,a,b] == t2[j,i,b,a]; t3[i,j,k,a,b,c]
    invariant under simultaneous permutations of the (i,a),(j,b),(k,c) columns
    (a Gaussian tensor averaged over the six column orderings).  Full tensors:
    small sizes only."""
    rng = np.random.default_rng(seed)
    t1 = rng.normal(0.0, scale1, (o, v))
    X2 = rng.normal(0.0, scale2, (o, o, v, v))
    t2 = 0.5 * (X2 + X2.transpose(1, 0, 3, 2))
    t3 = None
    if triples:
        X3 = rng.normal(0.0, scale3, (o, o, o, v, v, v))
        t3 = np.zeros_like(X3)
        for p in _col_perms(3):
            t3 += X3.transpose(p[0], p[1], p[2], 3 + p[0], 3 + p[1], 3 + p[2])
        t3 /= 6.0
    return t1, t2, t3


def packed_triples(o: int) -> list[tuple[int, int, int]]:
    """Occupied triples i <= j <= k in lexicographic order (the packed order)."""
    return [(i, j, k) for i in range(o) for j in range(i, o) for k in range(j, o)]


def random_t3_packed(o: int, v: int, seed: int, scale: float = 0.01, out: np.ndarray | None = None) -> np.ndarray:
    """Packed column-symmetric T3, shape (ntri, v, v, v), blocks in the order of
    :func:`packed_triples`.

    Block (i,j,k) is drawn from ``default_rng([seed, idx])`` so any block can be
    regenerated alone.  Blocks with equal occupied indices carry the symmetry
    that the column symmetry forces on them: i=j<k blocks are symmetric in the
    first two virtual axes, i<j=k blocks in the last two, i=j=k blocks in all
    three."""
    tri = packed_triples(o)
    if out is None:
        out = np.empty((len(tri), v, v, v))
    for idx, (i, j, k) in enumerate(tri):
        out[idx] = t3_block(v, seed, idx, (i, j, k), scale)
    return out


def t3_block(v: int, seed: int, idx: int, ijk: tuple[int, int, int], scale: float = 0.01) -> np.ndarray:
    """One block of :func:`random_t3_packed`."""
    i, j, k = ijk
    g = np.random.default_rng([seed, idx]).normal(0.0, scale, (v, v, v))
    if i == j == k:
        s = np.zeros_like(g)
        for p in _col_perms(3):
            s += g.transpose(p)
        s /= 6.0
        # read every element from its sorted index so the block is exactly symmetric
        a, b, c = np.meshgrid(np.arange(v), np.arange(v), np.arange(v), indexing="ij")
        srt = np.sort(np.stack([a, b, c]), axis=0)
        return s[srt[0], srt[1], srt[2]]
    if i == j:
        return 0.5 * (g + g.transpose(1, 0, 2))
    if j == k:
        return 0.5 * (g + g.transpose(0, 2, 1))
    return g


# ---------------------------------------------------------------------------
# Counter-based T3 for large sizes
# ---------------------------------------------------------------------------
# Element (block idx, flat offset e) of the packed T3 is a function of its
# global counter c = idx * v^3 + e alone: the SplitMix64 output function
# (Steele, Lea and Flood, OOPSLA 2014) applied to c and the seed gives a
# 64-bit word whose top 53 bits make a uniform double u in [0, 1); the value
# is scale * (2u - 1).  Any block can therefore be produced independently and
# in parallel, and a host can regenerate just the blocks it needs.

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _splitmix_uniform(counter: np.ndarray, seed: int) -> np.ndarray:
    z = counter + np.uint64(1)
    with np.errstate(over="ignore"):
        np.multiply(z, _GOLDEN, out=z)
        np.add(z, np.uint64((seed * 0xD1B54A32D192ED03) % (1 << 64)), out=z)
        np.bitwise_xor(z, z >> np.uint64(30), out=z)
        np.multiply(z, _M1, out=z)
        np.bitwise_xor(z, z >> np.uint64(27), out=z)
        np.multiply(z, _M2, out=z)
        np.bitwise_xor(z, z >> np.uint64(31), out=z)
    np.right_shift(z, np.uint64(11), out=z)
    return z.view(np.int64).astype(np.float64) * (1.0 / 9007199254740992.0)


def hashed_t3_block(v: int, seed: int, idx: int, ijk: tuple[int, int, int], scale: float = 0.01) -> np.ndarray:
    """Block idx = (i,j,k) of the counter-based packed T3, with the symmetry
    that equal occupied indices force (as in :func:`t3_block`)."""
    i, j, k = ijk
    v3 = v * v * v
    cnt = np.arange(v3, dtype=np.uint64) + np.uint64(idx * v3)
    g = (scale * (2.0 * _splitmix_uniform(cnt, seed) - 1.0)).reshape(v, v, v)
    if i == j == k:
        s = np.zeros_like(g)
        for p in _col_perms(3):
            s += g.transpose(p)
        s /= 6.0
        a, b, c = np.meshgrid(np.arange(v), np.arange(v), np.arange(v), indexing="ij")
        srt = np.sort(np.stack([a, b, c]), axis=0)
        return s[srt[0], srt[1], srt[2]]
    if i == j:
        return 0.5 * (g + g.transpose(1, 0, 2))
    if j == k:
        return 0.5 * (g + g.transpose(0, 2, 1))
    return g


def hashed_t3_packed(o: int, v: int, seed: int, scale: float = 0.01, out: np.ndarray | None = None,
                     threads: int = 8) -> np.ndarray:
    """Whole counter-based packed T3 (ntri, v, v, v), blocks filled in parallel."""
    from concurrent.futures import ThreadPoolExecutor

    tri = packed_triples(o)
    if out is None:
        out = np.empty((len(tri), v, v, v))

    def work(n):
        out[n] = hashed_t3_block(v, seed, n, tri[n], scale)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, range(len(tri))))
    return out


def hashed_t3_slab(o: int, v: int, seed: int, first: int, count: int, scale: float = 0.01,
                   threads: int = 8) -> np.ndarray:
    """Blocks [first, first + count) of the counter-based packed T3."""
    from concurrent.futures import ThreadPoolExecutor

    tri = packed_triples(o)
    out = np.empty((count, v, v, v))

    def work(m):
        out[m] = hashed_t3_block(v, seed, first + m, tri[first + m], scale)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, range(count)))
    return out


def hashed_uniform(shape, seed: int, scale: float = 0.1, threads: int = 8, chunk: int = 1 << 24) -> np.ndarray:
    """Array of the given shape with entries scale * U(-1, 1) from the
    counter-based generator (element n uses counter n), filled in parallel."""
    from concurrent.futures import ThreadPoolExecutor

    n = int(np.prod(shape))
    out = np.empty(n)

    def work(c0):
        c1 = min(n, c0 + chunk)
        cnt = np.arange(c0, c1, dtype=np.uint64)
        out[c0:c1] = scale * (2.0 * _splitmix_uniform(cnt, seed) - 1.0)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, range(0, n, chunk)))
    return out.reshape(shape)
