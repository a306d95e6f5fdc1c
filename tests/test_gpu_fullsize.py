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
