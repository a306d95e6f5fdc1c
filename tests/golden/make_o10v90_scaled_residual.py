"""Write o10v90_scaled_residual.txt: the oracle's residuals, element by
element, on the state after one iteration from the MP2 guess of the
variance-scaled o=10, v=90 workload (cct_inputs "o10v90-scaled").

After one iteration every T3 block with two or more distinct occupied indices
is non-zero (the T2 drivers fill it), so the residual exercises every R3 term, the
T3 feedback into R1/R2 and the T1 dressing at the measured shape.  Stored:
all of R1 (post-processed R3 as in Sec. "Removing redundancies in RCC
amplitudes"), 4000 sampled R2 elements and 7600 sampled R3 elements (2500
each from blocks with distinct indices, i=j<k, i<j=k, and 100 from i=j=k
blocks, which are exactly zero), with their indices.  Iteration 1 has a
single DIIS vector, so no extrapolation enters the state.

Calls only oracle/ and the input generator.  Needs about 50 GB of host
memory and two full residual evaluations (tens of minutes on an 8-core
host); run it alone.

  python tests/golden/make_o10v90_scaled_residual.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cct_inputs as ci  # noqa: E402
from oracle import rccsdt as R  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "o10v90_scaled_residual.txt")


def sample_r3_sites(o, v, rng):
    tri = R.packed_list(o)
    kinds = {
        "distinct": [t for t in tri if t[0] < t[1] < t[2]],
        "ij": [t for t in tri if t[0] == t[1] < t[2]],
        "jk": [t for t in tri if t[0] < t[1] == t[2]],
        "iii": [t for t in tri if t[0] == t[1] == t[2]],
    }
    counts = {"distinct": 2500, "ij": 2500, "jk": 2500, "iii": 100}
    sites = []
    for kind, n in counts.items():
        pool = kinds[kind]
        for _ in range(n):
            i, j, k = pool[int(rng.integers(len(pool)))]
            a, b, c = (int(x) for x in rng.integers(0, v, 3))
            sites.append((i, j, k, a, b, c))
    return sites


def main():
    s = ci.make_named("o10v90-scaled")
    o, v, f, B = s["o"], s["v"], s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS()
    print("iteration 1 ...", flush=True)
    t1, t2, t3, e1, _ = R.iterate(f, V, t1, t2, t3, o, diis=d, diis_t3="none")
    print(f"E after iteration 1: {e1!r}; residual ...", flush=True)
    r1, r2, r3 = R.residuals(f, V, t1, t2, t3, o)
    del t3
    r3 = R.postprocess_r3(r3)
    rng = np.random.default_rng(90210)
    lines = ["# Oracle residuals on the state after one iteration from the MP2 guess,",
             "# o=10 v=90 naux=200 seed 2, B entries N(0, 0.05 sqrt(48/naux)) (cct_inputs",
             "# o10v90-scaled), DIIS on T1/T2 only (no extrapolation in iteration 1).",
             "# Written by tests/golden/make_o10v90_scaled_residual.py (oracle only).",
             f"# energy_after_iteration_1 {float(e1)!r}",
             f"# max_abs R1 {float(np.abs(r1).max())!r} R2 {float(np.abs(r2).max())!r} R3 {float(np.abs(r3).max())!r}",
             "# rows: R1 i a value | R2 i j a b value | R3 i j k a b c value (i<=j<=k)"]
    for i in range(o):
        for a in range(v):
            lines.append(f"R1 {i} {a} {float(r1[i, a])!r}")
    for _ in range(4000):
        i, j, a, b = (int(x) for x in (rng.integers(o), rng.integers(o), rng.integers(v), rng.integers(v)))
        lines.append(f"R2 {i} {j} {a} {b} {float(r2[i, j, a, b])!r}")
    for (i, j, k, a, b, c) in sample_r3_sites(o, v, rng):
        lines.append(f"R3 {i} {j} {k} {a} {b} {c} {float(r3[i, j, k, a, b, c])!r}")
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
