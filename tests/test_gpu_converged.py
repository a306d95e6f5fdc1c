"""Converged energies in every precision mode (GPU, through the C ABI).

o=4, v=20 (seed 1): the oracle is iterated to a residual norm below 1e-10
(DIIS on T1, T2, T3); the GPU FP64 energy must agree within 1e-10 Eh and the
FP32 and split-BF16 energies within 1 microhartree.

o=10, v=90 (seed 2) with the variance-scaled integrals (the literal recipe
has no solution reachable from MP2 at this size): the full oracle is out of
reach of a test, so GPU FP64 (held to the oracle residual by residual in the
parity tests) converges to 1e-8 and is the reference for the mixed modes,
which must land within 1 microhartree of it.
"""

import sys

import numpy as np
import pytest

import cct_inputs as ci
from oracle import rccsdt as R
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _converge(s, o, v, naux, prec, tol, max_iter):
    with binding.Engine(o, v, naux, precision=prec) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        hist = []
        for it in range(max_iter):
            e, nr = eng.update()
            n = float(np.sqrt(nr.sum()))
            hist.append((e, n))
            if n < tol:
                break
    return hist


def test_converged_o4v20_all_modes_vs_oracle():
    o, v, naux, seed = ci.CONFIGS["o4v20"]
    s = ci.make_system(o, v, naux, seed)
    f, B = s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS()
    for it in range(200):
        t1, t2, t3, e_ref, nr = R.iterate(f, V, t1, t2, t3, o, diis=d)
        if np.sqrt(np.sum(nr)) < 1e-10:
            break
    say(f"[converged o4v20] oracle E={e_ref:.12f} after {it+1} iterations")
    for prec, tol_e in (("fp64", 1e-10), ("fp32", 1e-6), ("bf16x3", 1e-6)):
        hist = _converge(s, o, v, naux, prec, 1e-10 if prec == "fp64" else 1e-9, 200)
        e, n = hist[-1]
        say(f"  {prec}: E={e:.12f} |R|={n:.2e} after {len(hist)} iterations, dE={e - e_ref:.3e}")
        assert abs(e - e_ref) <= tol_e


def test_converged_o10v90_scaled_mixed_vs_fp64():
    s = ci.make_named("o10v90-scaled")
    o, v, naux = s["o"], s["v"], s["naux"]
    ref = _converge(s, o, v, naux, "fp64", 1e-8, 150)
    e_ref, n_ref = ref[-1]
    say(f"[converged o10v90-scaled] fp64 E={e_ref:.12f} |R|={n_ref:.2e} after {len(ref)} iterations")
    assert n_ref < 1e-8
    for prec in ("fp32", "bf16x3"):
        hist = _converge(s, o, v, naux, prec, 1e-8, len(ref) + 30)
        e, n = hist[-1]
        say(f"  {prec}: E={e:.12f} |R|={n:.2e} after {len(hist)} iterations, dE={e - e_ref:.3e}")
        assert abs(e - e_ref) <= 1e-6


def test_o10v90_first_iterations_match_oracle_golden():
    """The o=10 v=90 workload (variance-scaled integrals): energies and
    squared residual norms of the first three iterations from the MP2 guess
    against the oracle's values stored by
    tests/golden/make_o10v90_scaled_iterations.py (DIIS on T1/T2 only)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "o10v90_scaled_iterations.txt")
    rows = [list(map(float, ln.split())) for ln in open(path) if ln.strip() and not ln.startswith("#")]
    s = ci.make_named("o10v90-scaled")
    o, v, naux = s["o"], s["v"], s["naux"]
    print(f"[o10v90 golden] {len(rows)} iterations", flush=True)
    with binding.Engine(o, v, naux, opts={"diis_t3": "none"}) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        for it, e_ref, r1, r2, r3 in rows:
            e, nr = eng.update()
            print(f"  it {int(it)}: gpu {e:.14f} oracle {e_ref:.14f} diff {e - e_ref:.2e}", flush=True)
            assert abs(e - e_ref) < 1e-10
            for a, b in zip(nr, (r1, r2, r3)):
                assert abs(a - b) <= 1e-10 * max(1.0, b)


def test_o10v90_residual_elements_match_oracle_golden():
    """The o=10 v=90 workload (variance-scaled integrals), the residual on the
    state after one iteration from the MP2 guess, element by element against
    the oracle: all of R1, 4000 sampled R2 and 7600 sampled R3 elements
    (blocks with distinct indices, i=j<k, i<j=k, and i=j=k blocks, which must
    be exactly zero), stored by tests/golden/make_o10v90_scaled_residual.py.
    Tolerance: 1e-10 of the largest element of each residual."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "o10v90_scaled_residual.txt")
    if not os.path.exists(path):
        pytest.skip("golden residual file not written yet (tests/golden/make_o10v90_scaled_residual.py)")
    rows = {"R1": [], "R2": [], "R3": []}
    scale = {}
    for ln in open(path):
        if ln.startswith("# max_abs"):
            p = ln.split()
            scale = {p[2]: float(p[3]), p[4]: float(p[5]), p[6]: float(p[7])}
        if ln.strip() and not ln.startswith("#"):
            p = ln.split()
            rows[p[0]].append(([int(x) for x in p[1:-1]], float(p[-1])))
    s = ci.make_named("o10v90-scaled")
    o, v, naux = s["o"], s["v"], s["naux"]
    print(f"[o10v90 residual golden] {', '.join(f'{k}: {len(x)}' for k, x in rows.items())}", flush=True)
    with binding.Engine(o, v, naux, opts={"diis_t3": "none"}) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        eng.update()
        r1, r2, r3p, _ = eng.residual()
    tri = {t: n for n, t in enumerate(ci.packed_triples(o))}
    got = {"R1": [r1[i, a] for (i, a), _ in rows["R1"]],
           "R2": [r2[i, j, a, b] for (i, j, a, b), _ in rows["R2"]],
           "R3": [r3p[tri[(i, j, k)], a, b, c] for (i, j, k, a, b, c), _ in rows["R3"]]}
    for name in ("R1", "R2", "R3"):
        ref = np.array([x for _, x in rows[name]])
        g = np.array(got[name])
        err = float(np.abs(g - ref).max())
        print(f"  {name}: max err {err:.3e} of max |R| {scale[name]:.3e}", flush=True)
        assert err <= 1e-10 * scale[name]
    iii = [n for n, ((i, j, k, *_), _) in enumerate(rows["R3"]) if i == j == k]
    assert iii and all(got["R3"][n] == 0.0 for n in iii)
