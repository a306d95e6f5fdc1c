"""Write o10v90_scaled_iterations.txt: the oracle's energies and squared
residual norms for the first three iterations from the MP2 guess on the
variance-scaled o=10, v=90 workload (cct_inputs "o10v90-scaled"), with DIIS on
T1/T2 only (space 8, start 2; T3 takes plain Jacobi steps).

Calls only oracle/ and the input generator.  Needs about 50 GB of host
memory (the oracle works on the full 10^3 x 90^3 triples tensor and its
temporaries) and several minutes per iteration on an 8-core host; run it
alone.

  python tests/golden/make_o10v90_scaled_iterations.py
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cct_inputs as ci  # noqa: E402
from oracle import rccsdt as R  # noqa: E402


def main():
    s = ci.make_named("o10v90-scaled")
    o, f, B = s["o"], s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS()
    lines = ["# Oracle energies (Eh) and squared residual norms |R1|^2 |R2|^2 |R3|^2 (full-tensor)",
             "# after iterations 1..3 from the MP2 guess, o=10 v=90 naux=200 seed 2 with",
             "# B entries N(0, 0.05 sqrt(48/naux)) (cct_inputs o10v90-scaled); DIIS on T1/T2",
             "# only (space 8, start 2), T3 by Jacobi steps.  Written by",
             "# tests/golden/make_o10v90_scaled_iterations.py (oracle only).",
             "# columns: iteration energy r1 r2 r3"]
    for it in range(1, 4):
        t1, t2, t3, e, nrm = R.iterate(f, V, t1, t2, t3, o, diis=d, diis_t3="none")
        lines.append(f"{it} {e!r} {nrm[0]!r} {nrm[1]!r} {nrm[2]!r}")
        print(lines[-1], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "o10v90_scaled_iterations.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
