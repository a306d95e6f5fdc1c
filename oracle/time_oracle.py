"""Wall-clock timing of the FP64 CPU oracle (test infrastructure, host only).

Times one residual evaluation (all terms plus the R3 post-processing) and one
whole iteration (residual, Jacobi step, DIIS, energy) of `oracle.rccsdt` on the
named synthetic workloads, from the MP2 guess, median of `--repeat` runs, with
the BLAS/OpenMP thread count fixed before numpy is imported.  The batch
workload times one iteration of each of its 64 systems once and reports the
sum.  Prints one JSON line per workload.

  python -m oracle.time_oracle --workload o4v20 --threads 8
  python -m oracle.time_oracle --workload o10v90 --threads 8 --repeat 3
  python -m oracle.time_oracle --workload batch --threads 8
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True, choices=["o4v20", "o10v90", "batch"])
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    ap.add_argument("--repeat", type=int, default=3)
    ap.add_argument("--residual-only", action="store_true")
    args = ap.parse_args()
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = str(args.threads)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import numpy as np  # noqa: F401  (after the thread settings)

    import cct_inputs as ci
    from oracle import rccsdt as R

    def one(o, v, naux, seed):
        s = ci.make_system(o, v, naux, seed)
        f, V = s["f"], R.eri_phys_from_B(s["B"])
        t1, t2, t3 = R.mp2_guess(f, V, o)
        tr = time.perf_counter()
        r = R.residuals(f, V, t1, t2, t3, o)
        R.postprocess_r3(r[2])
        t_res = time.perf_counter() - tr
        t_it = None
        if not args.residual_only:
            ti = time.perf_counter()
            R.iterate(f, V, t1, t2, t3, o, diis=R.DIIS())
            t_it = time.perf_counter() - ti
        return t_res, t_it

    rec = {"workload": args.workload, "threads": args.threads, "cpu": _cpu_model(), "cores": os.cpu_count()}
    if args.workload == "batch":
        sizes = ci.batched_sizes()
        tres, tit = 0.0, 0.0
        for o, v, naux, seed in sizes:
            a, b = one(o, v, naux, seed)
            tres += a
            tit += b or 0.0
        rec.update({"systems": len(sizes), "s_per_residual_sum": tres,
                    "s_per_iteration_sum": tit if not args.residual_only else None,
                    "system_iterations_per_s": len(sizes) / tit if tit else None})
    else:
        o, v, naux, seed = ci.CONFIGS[args.workload]
        runs = [one(o, v, naux, seed) for _ in range(args.repeat)]
        rec.update({"o": o, "v": v, "naux": naux, "seed": seed, "repeat": args.repeat,
                    "s_per_residual_median": statistics.median(r[0] for r in runs),
                    "s_per_iteration_median": (statistics.median(r[1] for r in runs)
                                               if not args.residual_only else None)})
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
