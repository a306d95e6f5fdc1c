#!/usr/bin/env python3
"""Benchmark: one spin-restricted CCSDT iteration on compact T3 at o=20, v=180.

A step is one full iteration of the hot path (T1 dressing, RCCSD parts, T3
feedback, the whole triples residual R3 on packed i<=j<=k blocks,
post-processing, Jacobi update, DIIS on T1/T2, energy) on one MI355X, with all
inputs resident in device memory.  Prints one JSON line.

  value        R3 FLOP one iteration executes (2 x the compact multiply-add
               count, the ladder at its symmetric/antisymmetric count) / wall
               time of the step, TFLOP/s; value_direct_count uses the direct
               ladder count instead
  ms_per_step  seconds per CCSDT iteration x 1000
  roofline     the particle-particle ladder GEMMs (the dominant kernel):
               executed FLOP per launch / average launch time from HIP
               events on the library's stream, against the mode's matrix peak
  cpu_baseline the FP64 oracle on one sampled output block of the same
               workload, rate in the same unit
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cct_inputs as ci  # noqa: E402

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pp_ladder_gemm_o20v180_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(o, v, naux, seed):
    """Time the oracle on packed output blocks of the PP ladder (the dominant
    term) at the same sizes, about 10 s of work; report the algorithmic rate."""
    from oracle import blocks  # test infrastructure, CPU only
    from oracle import counts

    s = ci.make_system(o, v, naux, seed)
    B = s["B"]
    # MP2 amplitudes of this workload (the state the timed step starts from)
    Bov = B[:, :o, o:]
    vovov = np.einsum("Pia,Pjb->ijab", Bov, Bov, optimize=True)
    e = np.diag(s["f"])
    d2 = e[:o, None, None, None] + e[None, :o, None, None] - e[None, None, o:, None] - e[None, None, None, o:]
    t2 = vovov / d2
    t1 = np.zeros((o, v))
    tri = ci.packed_triples(o)
    idx = len(tri) // 2
    blk = ci.hashed_t3_block(v, 77, idx, tri[idx])
    Bt = blocks.dressed_factors(B, t1)
    t0 = time.time()
    W = blocks.w_vvvv(Bt, t2, o)
    t_w = time.time() - t0
    # time whole blocks (oracle work only, not their generation) until at
    # least 10 s have been spent, at most 12 blocks
    t_b = 0.0
    nblk = 0
    while t_b < 10.0 and nblk < 12:
        n = (idx + nblk) % len(tri)
        blk_n = blk if nblk == 0 else ci.hashed_t3_block(v, 77, n, tri[n])
        tb = time.time()
        r = blocks.postprocess_block(blocks.pp_block(W, blk_n, tri[n]), tri[n])
        t_b += time.time() - tb
        nblk += 1
        assert np.isfinite(r).all()
    # algorithmic FLOP of this sample in the metric's definition: the compact
    # particle-particle ladder work of one packed block (3 v^5 multiply-adds)
    flops = nblk * 2.0 * counts.r3_macs(o, v)["pp"] / counts.ntri(o)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {
        "value": flops / t_b / 1e12,
        "unit": "TFLOP/s",
        "cores": min(cores, threads),
        "kind": "oracle",
        "sample": (f"{nblk} packed blocks from (i,j,k)={tri[idx]} on of R3 (particle-particle ladder by its "
                   f"definition, 6 column permutations, + post-processing) at o={o} v={v}; {t_b:.1f} s; rate uses the "
                   f"compact per-block ladder work 3 v^5; W^ab_de build ({t_w:.1f} s) excluded"),
    }


NT_TILES = {0: "size-based", 1: "<128,256,2,4,2>", 2: "<256,128,4,2,2>", 3: "<64,64,2,2,2>", 4: "<128,128,2,2,2>",
            5: "<256,32,4,1,2>", 6: "<32,256,1,4,2>"}
LP_TILES = {"fp32": {0: "size-based", 1: "<128,128,2,2,1>", 2: "<128,128,2,4,2>", 3: "<64,64,2,2,2>"},
            "bf16x3": {0: "size-based", 1: "<256,128,4,2,1>", 2: "<128,128,2,4,2>", 3: "<64,64,2,2,2>",
                       4: "<256,256,2,4,1>"}}


def kernel_name(prec, variant):
    if prec == "fp64":
        return "gemm_nt_f64_kernel" + NT_TILES.get(variant, str(variant))
    return f"gemm_lp_{prec.replace('fp32', 'f32')}_kernel" + LP_TILES[prec].get(variant, str(variant))


def run_mode(binding, s, o, v, naux, prec, steps, warmup, tune_ms=0.0):
    """Warmup + timed iterations from the MP2 guess in one precision mode
    (tile variants autotuned first when tune_ms > 0, outside the timed steps)."""
    eng = binding.Engine(o, v, naux, precision=prec,
                         opts={"timers": True, "diis_t3": "none" if o >= 20 else "full"})
    try:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        variants = eng.autotune(tune_ms) if tune_ms > 0 else (0, 0)
        log(f"[bench] {prec}: tile variants ladder={variants[0]} rings={variants[1]}")
        # every cct_update ends with a synchronisation of the library's stream
        # (the energy and norms are read back), so the host clock brackets
        # exactly the device work of the timed steps.
        for w in range(warmup):
            e, nr = eng.update()
            log(f"[bench] {prec} warmup {w}: E={e:.10f}")
        phase_ms = {k: 0.0 for k in binding.PHASES}
        lad = {"ms": 0.0, "macs": 0.0, "launches": 0.0}
        t0 = time.perf_counter()
        for st in range(steps):
            e, nr = eng.update()
            macs, ms = eng.counters()
            for k in phase_ms:
                phase_ms[k] += ms[k]
            lad["ms"] += ms["ladder_gemm"]
            lad["macs"] += macs["ladder_gemm"]
            lad["launches"] += macs["ladder_launches"]
            log(f"[bench] {prec} step {st}: E={e:.10f} |R|={np.sqrt(nr.sum()):.3e}")
        wall = time.perf_counter() - t0
    finally:
        eng.close()
    term_macs = {k: macs[k] for k in binding.TERMS}
    # multiply-adds the step executes: the ladder at what its GEMMs ran (the
    # symmetric/antisymmetric form halves the direct count), the rest as counted
    r3_macs_direct = sum(term_macs.values())
    r3_macs = r3_macs_direct - term_macs["PP"] + lad["macs"] / steps
    r3_ms = sum(phase_ms[k] for k in ("pp", "rings", "hh_f2", "drivers", "f1")) / steps
    return {
        "ms_per_step": 1000.0 * wall / steps,
        "energy": e,
        "macs": term_macs,
        "r3_macs": r3_macs,
        "r3_macs_direct": r3_macs_direct,
        "r3_tflops": 2.0 * r3_macs / (r3_ms / 1000.0) / 1e12,
        "phase_ms": {k: x / steps for k, x in phase_ms.items()},
        "ladder_gemm": {"ms": lad["ms"] / steps, "macs": lad["macs"] / steps, "launches": lad["launches"] / steps},
        "tile_variants": {"ladder": variants[0], "rings": variants[1]},
    }


def run_batched(binding, niter, modes, tune_ms=0.0, graph=True, streams=4):
    """The 64-system batch (o uniform in 3..8, v in 20..60, seeded): niter
    iterations from the MP2 guess per mode, one graph replay per iteration.
    Rate: system-iterations per second over the timed iterations (the first,
    which records the graph, is excluded)."""
    sizes = ci.batched_sizes()
    # variance-scaled integrals: with sigma = 0.05 the largest members (naux up
    # to 136) diverge from the MP2 guess and their dE would measure chaos
    systems = [ci.make_system(o, v, na, seed, sigma=ci.scaled_sigma(na)) for o, v, na, seed in sizes]
    out = {}
    e_ref = None
    for prec in modes:
        with binding.Batch([(o, v, na) for o, v, na, _ in sizes], precision=prec,
                           opts={"graph": graph, "streams": streams}) as b:
            for k, s in enumerate(systems):
                b.set_system(k, s["f"], s["B"])
            if tune_ms > 0:
                b.autotune(tune_ms)
            b.iterate(1)
            t0 = time.perf_counter()
            e, nr = b.iterate(niter - 1)
            dt = time.perf_counter() - t0
        rec = {"systems_per_s": len(sizes) * (niter - 1) / dt, "s_per_batch_iteration": dt / (niter - 1)}
        if e_ref is None:
            e_ref = e
        else:
            d = e - e_ref
            rec["dE_max_abs"] = float(np.abs(d).max())
            rec["dE_rel_max"] = float(np.abs(d / e_ref).max())
        out[prec] = rec
        log(f"[bench] batched {prec}: {rec}")
    return {"workload": f"{len(sizes)} systems, o in [3,8], v in [20,60], naux=2(o+v), seeds 4000+s, "
                        "B entries N(0, 0.05 sqrt(48/naux)); "
                        f"{niter} iterations from MP2 (DIIS), first excluded from the rate",
            "unit": "system-iterations/s", "modes": out,
            "note": f"dE: energy after {niter} iterations minus the {modes[0]} batch's, per system"}


def run_accuracy(binding, modes, tol=1e-8, max_iter=150):
    """Converged energy per mode on o=10 v=90 with variance-scaled integrals
    (the named recipe has no solution reachable from MP2 at this size): FP64
    runs DIIS to |R| < tol; each other mode runs as many iterations; dE is
    measured against the FP64 energy."""
    s = ci.make_named("o10v90-scaled")
    o, v, naux = s["o"], s["v"], s["naux"]
    out = {"workload": "o=10 v=90 naux=200 seed 2, B entries N(0, 0.05 sqrt(48/naux)), DIIS on T1/T2/T3, "
                       f"FP64 to |R| < {tol:g}, other modes the same number of iterations"}
    e_ref, n_iter = None, max_iter
    for prec in modes:
        with binding.Engine(o, v, naux, precision=prec) as eng:
            eng.set_fock(s["f"])
            eng.set_eri_df(s["B"])
            eng.init_mp2()
            t0 = time.perf_counter()
            for it in range(n_iter):
                e, nr = eng.update()
                nrm = float(np.sqrt(nr.sum()))
                if e_ref is None and nrm < tol:
                    break
            wall = time.perf_counter() - t0
        rec = {"energy": e, "iterations": it + 1, "residual_norm": nrm, "s": wall}
        if e_ref is None:
            e_ref, n_iter = e, it + 1
        else:
            rec["dE"] = e - e_ref
        out[prec] = rec
        log(f"[bench] accuracy {prec}: {rec}")
    return out


SLAB = {"o": 50, "v": 400, "naux": 900, "seed": 5, "first": 0, "count": 64}


def run_slab(binding, modes, panel):
    """One process's share of a run sharded by packed triples: the block-local
    R3 terms (ladder with W^{ab}_{de} rebuilt in panels from the factors,
    F_vv term, T2 drivers, post-processing) for packed triples 0..63 at
    o=50, v=400, naux=900."""
    o, v, naux, seed = SLAB["o"], SLAB["v"], SLAB["naux"], SLAB["seed"]
    first, count = SLAB["first"], SLAB["count"]
    threads = min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8)
    t0 = time.time()
    s = ci.make_system(o, v, naux, seed)
    Bt = s["B"]  # T1 = 0: the dressed factors are the bare ones
    _, t2, _ = ci.random_amplitudes(o, v, seed, 0.0, 0.01, 0.0, triples=False)
    Fvv = ci.hashed_uniform((v, v), seed * 7 + 1, 0.1, threads)
    Wt = ci.hashed_uniform((o, v, v, v), seed * 7 + 2, 0.01, threads)
    Wvooo = ci.hashed_uniform((v, o, o, o), seed * 7 + 3, 0.01, threads)
    t3 = ci.hashed_t3_slab(o, v, seed, first, count, 0.01, threads)
    log(f"[bench] slab inputs ready in {time.time() - t0:.1f} s")
    out = {}
    for prec in modes:
        with binding.Slab(o, v, naux, first, count, precision=prec, opts={"panel": panel, "timers": True}) as sl:
            t1_ = time.time()
            sl.set_intermediates(Bt, t2, Fvv, Wt, Wvooo)
            sl.set_t3(t3)
            log(f"[bench] slab {prec}: inputs uploaded in {time.time() - t1_:.1f} s; residual ...")
            tr = time.perf_counter()
            _, n2 = sl.residual(want_r3=False)
            wall = time.perf_counter() - tr
            macs, ms = sl.counters()
        step_macs = macs["ladder"] + macs["f_vv"] + macs["driver_vvvo"] + macs["driver_vooo"]
        rec = {"s_per_residual": wall, "tflops": 2.0 * step_macs / wall / 1e12,
               "tflops_with_rebuild": 2.0 * (step_macs + macs["w_rebuild"]) / wall / 1e12,
               "ladder_tflops": 2.0 * macs["ladder"] / (ms["ladder"] / 1000.0) / 1e12,
               "peak": PEAK[prec], "phase_ms": ms, "norm2": n2}
        rec["ladder_frac"] = rec["ladder_tflops"] / PEAK[prec]
        out[prec] = rec
        log(f"[bench] slab {prec}: {rec}")
    return out


def q_macs(o, v):
    """Algorithmic multiply-adds of one E_(Q) evaluation in the occupied-tuple
    traversal: per ordered occupied tuple without three equal indices, the two
    contractions of v^5 (X from T3, Y from Wbar_ejk^abc), the two of o v^4 and
    the V outer product (v^4); plus the Wbar_ejk^abc build (2 o^2 v^5)."""
    nord = o ** 4 - o - 4 * o * (o - 1)
    return nord * (2 * v ** 5 + 2 * o * v ** 4 + v ** 4) + 2 * o * o * v ** 5


def q_cpu_baseline(s, t2, t3p, task=(0, 0, 1, 1)):
    """Time the one-tuple (Q) oracle on one task of the same workload and
    amplitudes (a bounded sample); rate with the GPU path's algorithmic count
    for the task's orderings."""
    from oracle import rccsdt as R, rccsdt_q as Q  # test infrastructure, CPU only
    import itertools

    o, v = s["o"], s["v"]
    V = R.eri_phys_from_B(s["B"])
    t3 = R.unpack_t3(t3p, o)
    t0 = time.time()
    e = Q.task_energy(s["f"], V, t2, t3, o, task)
    dt = time.time() - t0
    nq = len(set(itertools.permutations(task)))
    flop = 2.0 * nq * (2 * v ** 5 + 2 * o * v ** 4 + v ** 4)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": flop / dt / 1e12, "unit": "TFLOP/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": (f"task {task} ({nq} orderings) of E_(Q) at o={o} v={v}: {dt:.1f} s, energy {e:.6e}; rate uses "
                       f"the GPU path's count for these orderings (the oracle also rebuilds Wbar per ordering)")}


def run_q(binding, name, reps=2, cpu=True):
    """E_(Q) on a named workload after two FP64 iterations from the MP2 guess
    (T3 non-zero): wall time of cct_energy_q (setup of the intermediates and
    the task loop), algorithmic FLOP rate against the FP64 MFMA peak."""
    s = ci.make_named(name)
    o, v, naux = s["o"], s["v"], s["naux"]
    with binding.Engine(o, v, naux) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        for _ in range(2):
            eng.update()
        amps = eng.get_amplitudes() if cpu else None
        times, e = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            e = eng.energy_q()
            times.append(time.perf_counter() - t0)
            log(f"[bench] (Q) {name}: E_(Q) = {e:.12f} in {times[-1]:.2f} s")
    wall = min(times)
    flop = 2.0 * q_macs(o, v)
    out = {"workload": name, "e_q": e, "s": wall, "algorithmic_flop": flop, "tflops": flop / wall / 1e12,
           "peak": PEAK["fp64"], "frac": flop / wall / 1e12 / PEAK["fp64"]}
    if cpu:
        log("[bench] (Q) cpu baseline (oracle, one task) ...")
        out["cpu_baseline"] = q_cpu_baseline(s, amps[1], amps[2])
        log(f"[bench] (Q) cpu baseline: {out['cpu_baseline']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed iterations first (one makes T3 non-zero, so every term contracts real data)")
    ap.add_argument("--precision", default="fp64", choices=list(PEAK),
                    help="mode whose rate is the reported value")
    ap.add_argument("--compare", default="fp32,bf16x3",
                    help="further modes run from the same start for speedup and dE ('' for none)")
    ap.add_argument("--workload", default="o20v180", choices=list(ci.CONFIGS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune-ms", type=float, default=3000.0,
                    help="tile autotuning budget per mode before the timed steps (0: size-based defaults)")
    ap.add_argument("--batched-iters", type=int, default=5,
                    help="iterations of the 64-system batch per mode (0 skips it)")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the converged-energy comparison of the modes")
    ap.add_argument("--batched-graph", type=int, default=1, help="1: replay a recorded graph, 0: enqueue eagerly")
    ap.add_argument("--batched-streams", type=int, default=4, help="streams the batch's systems are spread over")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (reference for the HBM byte counters)")
    ap.add_argument("--slab", action="store_true",
                    help="only the block-local terms of a 64-triple slab at o=50 v=400 (FP32 and split-BF16)")
    ap.add_argument("--panel", type=int, default=8, help="W rows a per rebuilt panel (--slab)")
    ap.add_argument("--q-workload", default="o10v90-scaled", metavar="NAME",
                    help="also time the (Q) correction on this workload ('none' skips it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (the multi-GPU path is a "
                                   "design only, sharded by packed triples)"}))
        sys.exit(2)
    if args.calibrate_copy:
        import torch

        n = args.calibrate_copy // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        assert bool((b[-1] == 1.0).item())
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}), flush=True)
        return

    from paper_2607_00981_amd import binding

    if args.slab:
        modes = [m for m in ("fp32", "bf16x3") if m in [args.precision] + args.compare.split(",")]
        res = run_slab(binding, modes, args.panel)
        best = max(res, key=lambda m: res[m]["tflops"])
        r = res[best]
        ladder_ms = r["phase_ms"]["ladder"]
        print(json.dumps({
            "metric": "slab step (iv) TFLOP/s vs matrix peak, o=50 v=400, 64 packed triples",
            "value": r["tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1000.0 * r["s_per_residual"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": DTYPE[best], "data": "synthetic",
            "config": {"workload": "block-local R3 terms (ladder with W^ab_de rebuilt in panels, F_vv, T2 drivers, "
                                   "post-processing) for packed triples 0..63 of o=50 v=400 naux=900 seed 5",
                       "precision": best, "panel": args.panel},
            "modes": res,
            "roofline": {"bound": "mfma", "achieved": r["ladder_tflops"], "peak": r["peak"], "unit": "TFLOP/s",
                         "frac": r["ladder_frac"], "traffic": None,
                         "kernel": f"gemm_lp_{best.replace('fp32', 'f32')}_kernel (ladder GEMMs, "
                                   f"{ladder_ms:.0f} ms over all panels)"},
        }), flush=True)
        return

    o, v, naux, seed = ci.CONFIGS[args.workload]
    s = ci.make_system(o, v, naux, seed)
    log(f"[bench] o={o} v={v} naux={naux} seed={seed} precision={args.precision}")
    main_run = run_mode(binding, s, o, v, naux, args.precision, args.steps, args.warmup, args.autotune_ms)
    macs, phase_ms, ms_step, e = main_run["macs"], main_run["phase_ms"], main_run["ms_per_step"], main_run["energy"]
    value = 2.0 * main_run["r3_macs"] / (ms_step / 1000.0) / 1e12
    # dominant kernel: the particle-particle ladder GEMMs (executed FLOP and
    # device time of those launches alone, from HIP events on the library's
    # stream around each group of launches)
    lad = main_run["ladder_gemm"]
    achieved = 2.0 * lad["macs"] / (lad["ms"] / 1000.0) / 1e12 if lad["ms"] > 0 else None
    peak = PEAK[args.precision]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        try:
            tf = json.load(open(TRAFFIC_FILE))
            if (tf.get("precision") == args.precision and tf.get("workload") == args.workload and
                    tf.get("form") == "split" and tf.get("kernel") == kernel_name(args.precision,
                                                                                   main_run["tile_variants"]["ladder"])):
                traffic = tf.get("bytes_per_launch")
        except Exception:
            traffic = None
    modes = {args.precision: {"s_per_iteration": ms_step / 1000.0, "r3_tflops": main_run["r3_tflops"],
                              "energy": e, "speedup": 1.0, "dE": 0.0, "dE_rel": 0.0,
                              "tile_variants": main_run["tile_variants"]}}
    for prec in [m for m in args.compare.split(",") if m and m != args.precision]:
        r = run_mode(binding, s, o, v, naux, prec, args.steps, args.warmup, args.autotune_ms)
        modes[prec] = {"s_per_iteration": r["ms_per_step"] / 1000.0, "r3_tflops": r["r3_tflops"],
                       "energy": r["energy"], "speedup": ms_step / r["ms_per_step"],
                       "dE": r["energy"] - e, "dE_rel": (r["energy"] - e) / max(abs(e), 1e-300),
                       "phase_ms": r["phase_ms"], "tile_variants": r["tile_variants"]}
    out = {
        "metric": "T3-residual TFLOP/s + s/CCSDT iteration, FP64 vs mixed, o=20 v=180, dE vs oracle",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"RCCSDT iteration o={o} v={v} naux={naux} seed={seed}, compact T3 "
                               f"({o*(o+1)*(o+2)//6} triples x {v}^3), MP2 start, DIIS on T1/T2",
                   "precision": args.precision},
        "s_per_iteration": ms_step / 1000.0,
        "r3_tflops": main_run["r3_tflops"],
        "value_direct_count": 2.0 * main_run["r3_macs_direct"] / (ms_step / 1000.0) / 1e12,
        "phase_ms": phase_ms,
        "modes": modes,
        "modes_note": ("each mode runs warmup+steps iterations from the same MP2 guess (T3 = 0); dE = E(mode) - "
                       f"E({args.precision}) after the last step, exactly 0 for fewer than 3 iterations since the "
                       "mixed contractions act on T3, which reaches the energy two iterations later; converged "
                       "dE per mode: 'accuracy'"),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak if achieved else None, "traffic": traffic,
                     "kernel": kernel_name(args.precision, main_run["tile_variants"]["ladder"]) +
                               " (particle-particle ladder GEMMs)",
                     "launches_per_step": lad["launches"], "ms_per_launch": lad["ms"] / max(lad["launches"], 1),
                     "flop_per_launch": 2.0 * lad["macs"] / max(lad["launches"], 1)},
        "energy": e,
    }
    if args.batched_iters > 1:
        out["batched"] = run_batched(binding, args.batched_iters,
                                     [args.precision] + [m for m in args.compare.split(",") if m and m != args.precision],
                                     args.autotune_ms, bool(args.batched_graph), args.batched_streams)
    if not args.no_accuracy:
        out["accuracy"] = run_accuracy(binding, [args.precision] + [m for m in args.compare.split(",")
                                                                    if m and m != args.precision])
    if args.q_workload and args.q_workload != "none":
        log(f"[bench] (Q) correction on {args.q_workload} ...")
        out["q"] = run_q(binding, args.q_workload, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(o, v, naux, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
