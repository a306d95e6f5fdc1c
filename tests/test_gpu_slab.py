"""Slab of packed triples (cct_slab_*): the block-local R3 terms (ladder with
W^{ab}_{de} rebuilt in panels, F_vv term, both T2 drivers, post-processing)
against the block oracle, block by block.

Inputs: seeded system, T1-dressed factors, pair-symmetric T2, random
replicated intermediates (the terms are linear in them), counter-based T3.
Slabs start and end mid-list and include i=j<k, i<j=k and i=j=k blocks;
panels do not divide v (ragged last panel).  Tolerances as for the full
residual: 1e-11 (FP64), 2e-6 (FP32), 5e-5 (BF16X3) of the largest element
of the reference.
"""

import sys

import numpy as np
import pytest

import cct_inputs as ci
from oracle import blocks
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 2e-6, "bf16x3": 5e-5}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(o, v, naux, seed):
    rng = np.random.default_rng(seed)
    s = ci.make_system(o, v, naux, seed, sigma=0.1)
    t1, t2, _ = ci.random_amplitudes(o, v, seed, 0.03, 0.03, 0.0, triples=False)
    Bt = blocks.dressed_factors(s["B"], t1)
    Fvv = rng.normal(0, 0.1, (v, v))
    Wvvvo = rng.normal(0, 0.1, (v, v, v, o))  # [a][b][d][j]
    Wvooo = rng.normal(0, 0.1, (v, o, o, o))  # [a][l][i][j]
    t3p = ci.hashed_t3_packed(o, v, seed + 1, 0.02, threads=4)
    return Bt, t2, Fvv, Wvvvo, Wvooo, t3p


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("o,v,naux,first,count,panel", [(4, 12, 28, 3, 9, 5), (3, 11, 25, 1, 8, 4),
                                                         (2, 16, 36, 0, 4, 16)])
def test_slab_matches_block_oracle(prec, o, v, naux, first, count, panel):
    say(f"[slab parity] prec={prec} o={o} v={v} naux={naux} slab=[{first},{first + count}) panel={panel}")
    Bt, t2, Fvv, Wvvvo, Wvooo, t3p = _inputs(o, v, naux, 40 + o + v)
    tri = ci.packed_triples(o)
    W = blocks.w_vvvv(Bt, t2, o)
    term_sets = [("PP", "F1", "D1", "D2")] + ([("PP",), ("F1",), ("D1",), ("D2",)] if prec == "fp64" else [])
    with binding.Slab(o, v, naux, first, count, precision=prec, opts={"panel": panel}) as sl:
        sl.set_intermediates(Bt, t2, Fvv, np.ascontiguousarray(Wvvvo.transpose(3, 0, 1, 2)), Wvooo)
        sl.set_t3(t3p[first:first + count])
        for terms in term_sets:
            got, n2 = sl.residual(terms)
            ref = np.array([blocks.local_terms_block(W, Fvv, Wvvvo, Wvooo, t2, t3p[n], tri[n], terms=terms)
                            for n in range(first, first + count)])
            scale = max(float(np.abs(ref).max()), 1e-300)
            err = float(np.abs(got - ref).max())
            say(f"  terms={'+'.join(terms)}: max err {err:.3e} (scale {scale:.3e})")
            assert err <= TOL[prec] * scale
            mult = np.array([1 if i == j == k else (3 if (i == j or j == k) else 6)
                             for (i, j, k) in tri[first:first + count]], dtype=float)
            n2_ref = float(np.sum(mult[:, None, None, None] * ref * ref))
            assert abs(n2 - n2_ref) <= max(1e-10, 10 * TOL[prec]) * max(1.0, n2_ref)
