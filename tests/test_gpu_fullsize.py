"""Full-size parity at o=20, v=180, naux=400 (the bench workload), FP64.

The full-tensor oracle cannot hold T3 at this size (373 GB), so the check is
on sampled output blocks: the GPU evaluates the particle-particle ladder (the
dominant term, the one bench.py's roofline reports) with the same kernels and
launch configuration as a bench step, and oracle/blocks.py evaluates whole
packed blocks of it by definition (all six column permutations).  T3 is the
counter-based generator's (any block regenerable alone).  Sampled blocks cover
distinct, i=j<k, i<j=k and i=j=k triples and the first/last block.
Tolerance: 1e-11 of the block's largest element.
"""

import os
import sys
import time

import numpy as np
import pytest

import cct_inputs as ci
from oracle import blocks
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_pp_ladder_blocks_o20v180():
    o, v, naux, seed = ci.CONFIGS["o20v180"]
    s = ci.make_system(o, v, naux, seed)
    t1, t2, _ = ci.random_amplitudes(o, v, 77, 0.01, 0.01, 0.0, triples=False)
    tri = ci.packed_triples(o)
    t0 = time.time()
    say(f"[fullsize] generating packed T3 ({len(tri)} x {v}^3) ...")
    t3p = ci.hashed_t3_packed(o, v, 78, 0.01, threads=min(16, os.cpu_count() or 1))
    say(f"[fullsize] T3 ready in {time.time() - t0:.1f} s; GPU residual (PP) ...")
    sample = [0, tri.index((0, 1, 2)), tri.index((3, 3, 7)), tri.index((2, 9, 9)), tri.index((5, 5, 5)),
              tri.index((4, 11, 17)), len(tri) - 1]
    v3 = v ** 3
    with binding.Engine(o, v, naux, opts={"diis_t3": "none"}) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.set_amplitudes(t1, t2, t3p)
        del t3p
        t0 = time.time()
        eng.residual(["PP"], want_r3=False)
        say(f"[fullsize] GPU residual {time.time() - t0:.1f} s")
        got = {n: eng.copy_r3(n * v3, v3).reshape(v, v, v) for n in sample}
    t0 = time.time()
    W = blocks.w_vvvv(blocks.dressed_factors(s["B"], t1), t2, o)
    say(f"[fullsize] oracle W built in {time.time() - t0:.1f} s")
    for n in sample:
        ijk = tri[n]
        blk = ci.hashed_t3_block(v, 78, n, ijk, 0.01)
        ref = blocks.postprocess_block(blocks.pp_block(W, blk, ijk), ijk)
        scale = max(float(np.abs(ref).max()), 1e-300)
        err = float(np.abs(got[n] - ref).max())
        say(f"[fullsize] block {n} {ijk}: max|ref| {scale:.3e} max err {err:.3e}")
        if ijk[0] == ijk[1] == ijk[2]:
            assert np.abs(got[n]).max() == 0.0
        else:
            assert err <= 1e-11 * scale


def test_slab_o50v400_sampled_elements():
    """Slab of packed triples 0..63 at o=50, v=400, naux=900 (the slab
    measurement's shape, split-BF16 ladder, panels of 8 rows): sampled
    post-processed elements against the element-wise oracle (W^{ab}_{de}
    rows built on demand; the full W would be 205 GB).  Inputs: the named
    recipe's factors (T1 = 0), pair-symmetric T2, counter-based
    intermediates and T3.  Tolerance 1e-4 of the largest sampled value."""
    o, v, naux, seed = ci.CONFIGS["o50v400"]
    first, count = 0, 64
    threads = min(16, os.cpu_count() or 1)
    t0 = time.time()
    s = ci.make_system(o, v, naux, seed)
    Bt = s["B"]
    _, t2, _ = ci.random_amplitudes(o, v, seed, 0.0, 0.01, 0.0, triples=False)
    Fvv = ci.hashed_uniform((v, v), seed * 7 + 1, 0.1, threads)
    Wt = ci.hashed_uniform((o, v, v, v), seed * 7 + 2, 0.01, threads)
    Wvooo = ci.hashed_uniform((v, o, o, o), seed * 7 + 3, 0.01, threads)
    t3 = ci.hashed_t3_slab(o, v, seed, first, count, 0.01, threads)
    say(f"[slab fullsize] inputs in {time.time() - t0:.1f} s; GPU slab (bf16x3) ...")
    tri = ci.packed_triples(o)
    rng = np.random.default_rng(7)
    picks = {0: [(0, 0, 0), (3, 5, 7)], 1: [(0, 0, 1), (399, 17, 17), (5, 200, 399)], 50: [(1, 2, 3), (100, 100, 4)],
             63: [(398, 0, 211)]}
    for t in (17, 40):
        picks[t] = [tuple(int(x) for x in rng.integers(0, v, 3)) for _ in range(2)]
    v3 = v ** 3
    with binding.Slab(o, v, naux, first, count, precision="bf16x3", opts={"panel": 8}) as sl:
        sl.set_intermediates(Bt, t2, Fvv, Wt, Wvooo)
        sl.set_t3(t3)
        t0 = time.time()
        _, n2 = sl.residual(want_r3=False)
        say(f"[slab fullsize] GPU residual {time.time() - t0:.1f} s, norm2 {n2:.6e}")
        got = {t: [sl.copy_r3(t * v3 + a * v * v + b * v + c, 1)[0] for (a, b, c) in abcs]
               for t, abcs in picks.items()}
    t0 = time.time()
    G = blocks.occ_virt_gram(Bt, o)
    Wv = Wt.transpose(1, 2, 3, 0)  # W^{ab}_{dj} as a [a][b][d][j] view
    say(f"[slab fullsize] oracle setup {time.time() - t0:.1f} s")
    refs = {}
    for t, abcs in picks.items():
        refs[t] = blocks.local_terms_elements(Bt, t2, Fvv, Wv, Wvooo, t3[t - first], tri[t], abcs, G)
    scale = max(float(np.abs(r).max()) for r in refs.values())
    for t, abcs in picks.items():
        for (abc, g, r) in zip(abcs, got[t], refs[t]):
            say(f"  block {t} {tri[t]} {abc}: gpu {g:.9e} oracle {r:.9e}")
            if tri[t][0] == tri[t][1] == tri[t][2]:
                assert g == 0.0
            else:
                assert abs(g - r) <= 1e-4 * scale


MIXED_TOL_FULL = {"fp32": 2e-6, "bf16x3": 5e-5}


@pytest.mark.timeout(900)
def test_mixed_modes_o20v180_ladder_and_ring_blocks():
    """FP32 and split-BF16 at the contraction lengths of the o=20 v=180
    workload (split ladder K = v(v+1)/2 = 16290 accumulated in FP32, ring
    K = o v = 3600): the particle-particle ladder and all three ring types
    (term mask PP|RA|RB|RC) on the same amplitudes in the three modes, the
    same launch configuration as the benchmark's steps; sampled packed blocks
    of the mixed modes against GPU FP64 (itself held to the block oracle for
    the ladder above and to the full oracle at smaller sizes).  Tolerance:
    2e-6 (FP32) and 5e-5 (split-BF16) of the largest FP64 element of the
    sampled blocks, as at the smaller parity shapes."""
    o, v, naux, seed = ci.CONFIGS["o20v180"]
    s = ci.make_named("o20v180-scaled")
    t1, t2, _ = ci.random_amplitudes(o, v, 79, 0.01, 0.01, 0.0, triples=False)
    tri = ci.packed_triples(o)
    t0 = time.time()
    say(f"[fullsize mixed] generating packed T3 ({len(tri)} x {v}^3) ...")
    t3p = ci.hashed_t3_packed(o, v, 80, 0.01, threads=min(16, os.cpu_count() or 1))
    say(f"[fullsize mixed] T3 ready in {time.time() - t0:.1f} s")
    sample = [0, tri.index((0, 1, 2)), tri.index((3, 3, 7)), tri.index((2, 9, 9)), tri.index((5, 5, 5)),
              tri.index((4, 11, 17)), len(tri) - 1]
    v3 = v ** 3
    got = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        with binding.Engine(o, v, naux, precision=prec, opts={"diis_t3": "none"}) as eng:
            eng.set_fock(s["f"])
            eng.set_eri_df(s["B"])
            eng.set_amplitudes(t1, t2, t3p)
            t0 = time.time()
            eng.residual(["PP", "RA", "RB", "RC"], want_r3=False)
            say(f"[fullsize mixed] {prec}: residual (PP + rings) {time.time() - t0:.1f} s")
            got[prec] = {n: eng.copy_r3(n * v3, v3) for n in sample}
    del t3p
    scale = max(float(np.abs(b).max()) for b in got["fp64"].values())
    assert scale > 0.0
    for prec, tol in MIXED_TOL_FULL.items():
        err = max(float(np.abs(got[prec][n] - got["fp64"][n]).max()) for n in sample)
        say(f"[fullsize mixed] {prec}: max |R3 - R3(fp64)| = {err:.3e} = {err / scale:.2e} of max |R3| {scale:.3e}")
        assert err <= tol * scale
        assert np.abs(got[prec][tri.index((5, 5, 5))]).max() == 0.0
