#!/usr/bin/env python3
"""Benchmark: one spin-restricted CCSDT iteration on compact T3 at o=20, v=180.

A step is one full iteration of the hot path (T1 dressing, RCCSD parts, T3
feedback, the whole triples residual R3 on packed i<=j<=k blocks,
post-processing, Jacobi update, DIIS on T1/T2, energy) on one MI355X, with all
inputs resident in device memory.  Prints one JSON line.

Workload: o=20 v=180 naux=400 seed 3 with the density-fitting entries drawn at
standard deviation 0.05 sqrt(48/400) (the variance-scaled variant of the named
recipe: the same shapes and the same work per iteration).  With 0.05 the
energy overflows within five iterations from the MP2 guess; with the scaled
entries it stays finite, while the residual norm still grows about tenfold per
iteration (DIIS on T1/T2 only), so that the budgeted run (at most about ten
iterations) works on finite data throughout.  Each mode starts from the MP2
guess.

Wall budget.  The run is capped by --budget-s (wall seconds from the start of
the process).  The main mode always runs one untimed iteration (T3 non-zero
from then on) and at least one timed one; the number of timed steps is the
requested one or as many as fit the main mode's share of the budget, and the
further requested warm-up iterations run (before the timed steps) only if the
budget has room for them beyond those.
"steps" and "warmup" report what ran; "steps_requested" and
"warmup_requested" what was asked.  The comparison modes, the batch and the
optional legs run within what is left and are skipped (and named in
"skipped") when their estimate does not fit.

  value        R3 FLOP one iteration executes (2 x the compact multiply-add
               count, the ladder at its symmetric/antisymmetric count) / wall
               time of the step, TFLOP/s; value_direct_count uses the direct
               ladder count instead
  ms_per_step  seconds per CCSDT iteration x 1000 (mean over timed steps)
  roofline     the particle-particle ladder GEMMs (the dominant kernel):
               executed FLOP per launch / average launch time from HIP
               events on the library's stream, against the mode's matrix peak
  cpu_baseline the FP64 oracle on sampled output blocks of the ladder at the
               same sizes, rate on the same FLOP basis as value
  modes        per precision mode: seconds per iteration, speedup over the
               main mode, max |R3(mode) - R3(main)| / max |R3(main)| on
               sampled packed blocks of the residual evaluated on the state
               after one iteration (identical in every mode: T3 = 0 at the
               MP2 guess, so the mixed contractions first act in iteration
               2), and E(mode) - E(main) after the third iteration
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

_now = time.perf_counter  # the clock of every budget decision and timed step
T_START = _now()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cct_inputs as ci  # noqa: E402

PEAK = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0 / 3.0}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3"}
# seconds per iteration relative to FP64 (measured at o=20 v=180), for
# budgeting the comparison modes before they run
REL_COST = {"fp64": 1.0, "fp32": 0.75, "bf16x3": 0.4}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pp_ladder_gemm_o20v180_traffic.json")
# packed triples whose R3 blocks are compared between modes (distinct,
# repeated first pair, repeated last pair, first and last blocks)
SAMPLE_TRIPLES = ((0, 0, 1), (0, 1, 2), (0, 1, 1), (3, 7, 11), (5, 9, 9), (17, 18, 19), (18, 18, 19))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elapsed():
    return _now() - T_START


# ---------------------------------------------------------------------------
# budget logic (host only)
# ---------------------------------------------------------------------------
def plan_steps(requested: int, per_step_s: float, available_s: float) -> int:
    """Timed steps that fit available_s at per_step_s each: at least one (the
    metric needs a measurement), at most the requested count."""
    if requested <= 0:
        return 0
    if per_step_s <= 0:
        return requested
    return max(1, min(requested, int(math.floor(available_s / per_step_s))))


def plan_extra_warmup(requested_extra: int, per_step_s: float, available_s: float) -> int:
    """Further untimed iterations (beyond the first) that fit what the timed
    steps leave; none when the budget is spent."""
    if requested_extra <= 0 or per_step_s <= 0:
        return max(0, requested_extra) if per_step_s <= 0 else 0
    return max(0, min(requested_extra, int(math.floor(available_s / per_step_s))))


def compare_reserve(modes, t_iter_main: float, setup_s: float, iters: int = 3, rel=None) -> float:
    """Estimated seconds for the comparison modes: setup plus `iters`
    iterations each, scaled from the main mode's iteration time."""
    rel = rel or REL_COST
    return sum(setup_s + iters * rel.get(m, 1.0) * t_iter_main for m in modes)


def sample_offsets(o: int, v: int):
    """(triple, first element, count) of the sampled packed R3 blocks that exist at this o."""
    out = []
    for ijk in SAMPLE_TRIPLES:
        if max(ijk) < o:
            t = ci.packed_triples(o).index(tuple(ijk))
            out.append((tuple(ijk), t * v ** 3, v ** 3))
    seen, uniq = set(), []
    for rec in out:
        if rec[1] not in seen:
            seen.add(rec[1])
            uniq.append(rec)
    return uniq


def ladder_split_macs_per_block(v: int) -> float:
    """Multiply-adds of the symmetric/antisymmetric ladder per packed block:
    three terms, each v free virtuals x v(v+1)/2 output pairs x (v(v+1)/2 +
    v(v-1)/2) = v^2 summed pairs."""
    p = v * (v + 1) / 2.0
    return 3.0 * v * p * v * v


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on sampled blocks
# ---------------------------------------------------------------------------
def cpu_baseline(s, budget_s=10.0, max_blocks=12):
    """Time the oracle on packed output blocks of the PP ladder (the dominant
    term) at the same sizes, about budget_s of work; report the rate on the
    main value's basis (the split ladder's executed count) and on the direct
    count."""
    from oracle import blocks  # test infrastructure, CPU only

    o, v, B = s["o"], s["v"], s["B"]
    # MP2 amplitudes of this workload (the state the iteration starts from)
    Bov = B[:, :o, o:]
    vovov = np.einsum("Pia,Pjb->ijab", Bov, Bov, optimize=True)
    e = np.diag(s["f"])
    d2 = e[:o, None, None, None] + e[None, :o, None, None] - e[None, None, o:, None] - e[None, None, None, o:]
    t2 = vovov / d2
    t1 = np.zeros((o, v))
    tri = ci.packed_triples(o)
    idx = len(tri) // 2
    Bt = blocks.dressed_factors(B, t1)
    t0 = time.time()
    W = blocks.w_vvvv(Bt, t2, o)
    t_w = time.time() - t0
    t_b, nblk = 0.0, 0
    while t_b < budget_s and nblk < max_blocks:
        n = (idx + nblk) % len(tri)
        blk_n = ci.hashed_t3_block(v, 77, n, tri[n])
        tb = time.time()
        r = blocks.postprocess_block(blocks.pp_block(W, blk_n, tri[n]), tri[n])
        t_b += time.time() - tb
        nblk += 1
        assert np.isfinite(r).all()
    del W
    flops_split = nblk * 2.0 * ladder_split_macs_per_block(v)
    flops_direct = nblk * 2.0 * 3.0 * v ** 5
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {
        "value": flops_split / t_b / 1e12,
        "unit": "TFLOP/s",
        "cores": min(cores, threads),
        "kind": "oracle",
        "value_direct_count": flops_direct / t_b / 1e12,
        "sample": (f"{nblk} packed blocks from (i,j,k)={tri[idx]} on of R3 (particle-particle ladder by its "
                   f"definition, 6 column permutations, + post-processing) at o={o} v={v}; {t_b:.1f} s of oracle "
                   f"work; value counts the split ladder's 1.5 v^4 (v+1) multiply-adds per block (the basis of the "
                   f"GPU value), value_direct_count the direct 3 v^5; W^ab_de build ({t_w:.1f} s) excluded"),
    }


# ---------------------------------------------------------------------------
# one precision mode
# ---------------------------------------------------------------------------
NT_TILES = {0: "size-based", 1: "<128,256,2,4,2>", 2: "<256,128,4,2,2>", 3: "<64,64,2,2,2>", 4: "<128,128,2,2,2>",
            5: "<256,32,4,1,2>", 6: "<32,256,1,4,2>"}
LP_TILES = {"fp32": {0: "size-based", 1: "<128,128,2,2,1>", 2: "<128,128,2,4,2>", 3: "<64,64,2,2,2>"},
            "bf16x3": {0: "size-based", 1: "<256,128,4,2,1>", 2: "<128,128,2,4,2>", 3: "<64,64,2,2,2>",
                       4: "<256,256,2,4,1>"}}
# tile variants whose operand tiles are copied straight into LDS (their own kernels)
DL_KERNELS = {("fp64", 9): "gemm_nt_f64_dl_kernel<128,256,2,4>", ("fp64", 10): "gemm_nt_f64_dl_kernel<192,256,2,4>",
              ("fp64", 11): "gemm_nt_f64_dl_kernel<128,192,2,4>",
              ("bf16x3", 5): "gemm_lp_bf16x3_dl_kernel<256,256,2,4>", ("fp32", 5): "gemm_lp_f32_dl_kernel<128,128,2,4,2>"}


def kernel_name(prec, variant):
    if (prec, variant) in DL_KERNELS:
        return DL_KERNELS[(prec, variant)]
    if prec == "fp64":
        return "gemm_nt_f64_kernel" + NT_TILES.get(variant, str(variant))
    return f"gemm_lp_{prec.replace('fp32', 'f32')}_kernel" + LP_TILES[prec].get(variant, str(variant))


def run_mode(binding, s, prec, steps, warmup, tune_ms, samples, end_of, *, main=True):
    """One precision mode from the MP2 guess: autotune (outside the timed
    steps), one untimed iteration, then timed iterations.  end_of(t_it) gives
    the wall time (seconds from the start of the process) by which the mode
    should be done, from its iteration time.  Main mode: the requested number
    of timed steps or as many as fit (at least one), preceded by the remaining
    requested warm-ups if the budget has room for them too.  Comparison mode:
    up to `steps` timed iterations while the next one fits.  Every cct_update ends with a
    synchronisation of the library's stream (energy and norms are read back),
    so the host clock around each call brackets exactly its device work.
    After the second iteration overall the sampled R3 blocks (the residual of
    the state after one iteration) are copied out, outside any timing."""
    o, v, naux = s["o"], s["v"], s["naux"]
    t_setup0 = _now()
    eng = binding.Engine(o, v, naux, precision=prec,
                         opts={"timers": True, "diis_t3": "none" if o >= 20 else "full"})
    energies, norms, step_s = [], [], []
    r3_samples = None
    phase_ms = {k: 0.0 for k in binding.PHASES}
    lad = {"ms": 0.0, "macs": 0.0, "launches": 0.0}
    macs = None
    try:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        variants = eng.autotune(tune_ms) if tune_ms > 0 else (0, 0)
        setup_s = _now() - t_setup0
        log(f"[bench] {prec}: setup {setup_s:.1f} s, tile variants ladder={variants[0]} rings={variants[1]}")

        def iterate(tag):
            nonlocal r3_samples
            t0 = _now()
            e, nr = eng.update()
            dt = _now() - t0
            energies.append(e)
            norms.append(float(np.sqrt(nr.sum())))
            log(f"[bench] {prec} {tag}: E={e:.12f} |R|={norms[-1]:.3e} {dt:.2f} s (t={elapsed():.0f} s)")
            if len(energies) == 2 and samples:
                r3_samples = [eng.copy_r3(first, count) for _, first, count in samples]
            return dt

        def timed_step(k):
            nonlocal macs
            step_s.append(iterate(f"step {k}"))
            macs, ms = eng.counters()
            for key in phase_ms:
                phase_ms[key] += ms[key]
            lad["ms"] += ms["ladder_gemm"]
            lad["macs"] += macs["ladder_gemm"]
            lad["launches"] += macs["ladder_launches"]

        warm_done = 0
        if warmup > 0:
            # the first iteration (from T3 = 0) runs a few per cent faster than
            # later ones; the estimate is padded accordingly
            t_it = 1.05 * iterate("warmup 0")
            warm_done = 1
        else:
            timed_step(0)
            t_it = step_s[0]
        end = end_of(t_it)
        todo = steps - len(step_s)
        if main:
            n_steps = plan_steps(todo, t_it, end - elapsed()) if todo > 0 else 0
            extra = plan_extra_warmup(warmup - warm_done, t_it, end - elapsed() - n_steps * t_it)
            log(f"[bench] {prec}: ~{t_it:.2f} s per iteration; {n_steps + len(step_s)} timed steps of {steps} "
                f"and {warm_done + extra} warm-up iterations of {warmup} requested fit the mode's budget "
                f"(ends at t={end:.0f} s)")
            for k in range(extra):
                iterate(f"warmup {warm_done + k}")
            warm_done += extra
            for k in range(n_steps):
                timed_step(len(step_s))
        else:
            for k in range(max(todo, 1 if not step_s else 0)):
                if step_s and elapsed() + t_it > end:
                    break
                timed_step(len(step_s))
    finally:
        eng.close()
    n = len(step_s)
    term_macs = {k: macs[k] for k in binding.TERMS}
    # multiply-adds the step executes: the ladder at what its GEMMs ran (the
    # symmetric/antisymmetric form halves the direct count), the rest as counted
    r3_macs_direct = sum(term_macs.values())
    r3_macs = r3_macs_direct - term_macs["PP"] + lad["macs"] / n
    r3_ms = sum(phase_ms[k] for k in ("pp", "rings", "hh_f2", "drivers", "f1")) / n
    return {
        "steps": n, "warmup": warm_done, "setup_s": setup_s, "ms_per_step": 1000.0 * sum(step_s) / n,
        "step_s": step_s, "energies": energies, "norms": norms, "energy": energies[-1], "macs": term_macs,
        "r3_macs": r3_macs, "r3_macs_direct": r3_macs_direct,
        "r3_tflops": 2.0 * r3_macs / (r3_ms / 1000.0) / 1e12,
        "phase_ms": {k: x / n for k, x in phase_ms.items()},
        "ladder_gemm": {"ms": lad["ms"] / n, "macs": lad["macs"] / n, "launches": lad["launches"] / n},
        "tile_variants": {"ladder": variants[0], "rings": variants[1]}, "r3_samples": r3_samples,
    }


def r3_deviation(ref, got):
    """max |got - ref| / max |ref| over the sampled blocks."""
    if ref is None or got is None:
        return None
    num = max(float(np.abs(g - r).max()) for r, g in zip(ref, got))
    den = max(float(np.abs(r).max()) for r in ref)
    return num / den if den > 0 else None


# ---------------------------------------------------------------------------
# optional legs
# ---------------------------------------------------------------------------
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
            for k, sy in enumerate(systems):
                b.set_system(k, sy["f"], sy["B"])
            if tune_ms > 0:
                b.autotune(tune_ms)
            b.iterate(1)
            t0 = _now()
            e, nr = b.iterate(niter - 1)
            dt = _now() - t0
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


def run_accuracy(binding, modes, tol=1e-8, max_iter=150, workload="o10v90-scaled", iters=None, ref_energy=None):
    """Converged energy per mode: the first mode runs DIIS to |R| < tol (or
    exactly `iters` iterations); each other mode runs as many iterations; dE
    is measured against the first mode's energy, or against `ref_energy`
    (an FP64 energy after the same number of iterations from an earlier run)."""
    s = ci.make_named(workload)
    o, v, naux = s["o"], s["v"], s["naux"]
    base, _, variant = workload.partition("-")
    sigma = ci.variant_sigma(variant, naux)
    stop = f"exactly {iters} iterations" if iters else f"the first mode to |R| < {tol:g}"
    # T3 in the DIIS history needs 8 stored copies of it: from o = 20 on, T1/T2 only
    diis_t3 = "none" if o >= 20 else "full"
    out = {"workload": f"o={o} v={v} naux={naux} seed {s['seed']}, B entries N(0, {sigma:.6g}), DIIS on "
                       f"{'T1/T2' if diis_t3 == 'none' else 'T1/T2/T3'}, {stop}, other modes the same number of "
                       "iterations"}
    e_ref, n_iter = ref_energy, iters or max_iter
    fixed = iters is not None or ref_energy is not None
    for prec in modes:
        traj = []
        with binding.Engine(o, v, naux, precision=prec, opts={"diis_t3": diis_t3}) as eng:
            eng.set_fock(s["f"])
            eng.set_eri_df(s["B"])
            eng.init_mp2()
            t0 = _now()
            for it in range(n_iter):
                e, nr = eng.update()
                nrm = float(np.sqrt(nr.sum()))
                traj.append((e, nrm))
                log(f"[bench] converge {prec}: iteration {it + 1} E={e:.12f} |R|={nrm:.3e} ({_now() - t0:.1f} s)")
                if not fixed and e_ref is None and nrm < tol:
                    break
            wall = _now() - t0
        rec = {"energy": e, "iterations": it + 1, "residual_norm": nrm, "s": wall,
               "energies": [x for x, _ in traj], "residual_norms": [y for _, y in traj]}
        if e_ref is None:
            e_ref, n_iter = e, it + 1
        else:
            rec["dE"] = e - e_ref
        out[prec] = rec
        log(f"[bench] accuracy {prec}: energy {e!r} after {it + 1} iterations, |R| {nrm:.3e}")
    if ref_energy is not None:
        out["reference_energy"] = ref_energy
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
            tr = _now()
            _, n2 = sl.residual(want_r3=False)
            wall = _now() - tr
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


QUAD = {"o": 6, "v": 48, "seed": 11}


def run_quad(binding, modes, o=None, v=None):
    """The quadruples ladder on compact T4 (the RCCSDTQ quadruples
    residual's leading O(o^4 v^6) term in its six-term compact form): one
    evaluation per mode on random symmetric W and column-symmetric T4 blocks,
    algorithmic rate 2 x 6 nq v^6 / GEMM time and / wall time."""
    o = o or QUAD["o"]
    v = v or QUAD["v"]
    nq = binding.quad_count(o)
    rng = np.random.default_rng(QUAD["seed"])
    W = rng.normal(0.0, 0.1, (v, v, v, v))
    W = 0.5 * (W + W.transpose(1, 0, 3, 2))
    t4p = rng.normal(0.0, 0.01, (nq, v, v, v, v))
    out = {"workload": f"o={o} v={v}: {nq} stored blocks x {v}^4, W^ab_ef random (W^ab_ef = W^ba_fe), "
                       f"T4 blocks random", "modes": {}}
    for prec in modes:
        with binding.Quad(o, v, precision=prec, opts={"timers": True}) as q:
            q.set(W, t4p)
            q.ladder(want_r4=False)  # warm-up
            t0 = _now()
            q.ladder(want_r4=False)
            wall = _now() - t0
            macs, ms = q.counters()
        flop = 2.0 * macs["ladder"]
        rec = {"s": wall, "gemm_ms": ms["gemm"], "relabel_ms": ms["relabel"], "flop": flop,
               "tflops_wall": flop / wall / 1e12, "tflops_gemm": flop / (ms["gemm"] / 1000.0) / 1e12,
               "peak": PEAK[prec]}
        rec["frac_gemm"] = rec["tflops_gemm"] / PEAK[prec]
        out["modes"][prec] = rec
        log(f"[bench] quad {prec}: {rec}")
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
            t0 = _now()
            e = eng.energy_q()
            times.append(_now() - t0)
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


QABC = {"workload": "o20v180-weak", "block": 6, "ntasks": 24}


def run_q_abc(binding, name, block, ntasks):
    """E_(Q) in the virtual-tuple order on a sample of its tasks (tile
    quadruples spread evenly over the task list) at the state after one
    iteration from MP2: device time of the one-time set-up (integral slices
    and the T3 transposition) and of the sampled tasks, the executed
    matrix-core rate, and the full evaluation's time extrapolated from the
    sample."""
    s = ci.make_named(name)
    o, v, naux = s["o"], s["v"], s["naux"]
    ntot = binding.q_abc_task_count(v, block)
    n = min(ntasks, ntot)
    pick = sorted(set(int(round(k * (ntot - 1) / max(n - 1, 1))) for k in range(n)))
    with binding.Engine(o, v, naux, precision="bf16x3", opts={"diis_t3": "none" if o >= 20 else "full"}) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        eng.update()
        log(f"[bench] (Q) virtual-tuple order on {name}: {len(pick)} of {ntot} tasks, block {block} ...")
        t0 = _now()
        res = eng.energy_q_abc(block, tasks=pick)
        wall = _now() - t0
    st = res["stats"]
    tasks_s = st["tasks_ms"] / 1000.0
    rate = 2.0 * st["mfma_macs"] / tasks_s / 1e12 if tasks_s > 0 else None
    out = {"workload": f"{name} (o={o} v={v} naux={naux}), T2/T3 after one iteration from MP2",
           "block": block, "tasks_total": ntot, "tasks_timed": len(pick), "e_q_sampled_tasks": res["e_q"],
           "wall_s": wall, "setup_s": st["setup_ms"] / 1000.0, "tasks_s": tasks_s,
           "s_per_task": tasks_s / len(pick), "mfma_flop": 2.0 * st["mfma_macs"], "valu_flop": 2.0 * st["valu_macs"],
           "tflops_mfma_over_tasks": rate, "peak": PEAK["fp64"], "frac": rate / PEAK["fp64"] if rate else None,
           "full_evaluation_s_extrapolated": st["setup_ms"] / 1000.0 + tasks_s * ntot / len(pick)}
    log(f"[bench] (Q) virtual-tuple order: {out}")
    return out


# ---------------------------------------------------------------------------
def stored_traffic(prec, workload, kernel):
    """HBM bytes per launch of the ladder GEMM from the committed counter
    summary, when it was taken on this mode, workload and kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        tf = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if (tf.get("precision") == prec and tf.get("workload") == workload.split("-")[0] and tf.get("form") == "split"
            and tf.get("kernel") == kernel):
        return tf.get("bytes_per_launch")
    return None


def main(argv=None, binding=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed iterations (the first one makes T3 non-zero, so every term contracts real data)")
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall seconds for the whole run, counted from the start of the process")
    ap.add_argument("--precision", default="fp64", choices=list(PEAK),
                    help="mode whose rate is the reported value")
    ap.add_argument("--compare", default="bf16x3,fp32",
                    help="further modes run from the same start for speedup, R3 deviation and dE ('' for none)")
    ap.add_argument("--compare-steps", type=int, default=2,
                    help="timed iterations per comparison mode (after its untimed first one)")
    ap.add_argument("--workload", default="o20v180-scaled",
                    help="named workload (o4v20, o10v90, o20v180; '-scaled' for the variance-scaled integrals)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="oracle work timed for cpu_baseline")
    ap.add_argument("--autotune-ms", type=float, default=3000.0,
                    help="tile autotuning budget per mode before the timed steps (0: size-based defaults)")
    ap.add_argument("--batched-iters", type=int, default=5,
                    help="iterations of the 64-system batch per mode (0 skips it)")
    ap.add_argument("--accuracy", action="store_true",
                    help="also the converged-energy comparison of the modes on o10v90-scaled")
    ap.add_argument("--converge", default=None, metavar="NAME",
                    help="only the converged-energy comparison of the modes on this workload (e.g. o20v180-weak)")
    ap.add_argument("--converge-tol", type=float, default=1e-7, help="|R| at which the first mode stops")
    ap.add_argument("--converge-max-iter", type=int, default=40)
    ap.add_argument("--converge-iters", type=int, default=None,
                    help="run exactly this many iterations in every mode")
    ap.add_argument("--converge-ref-energy", type=float, default=None,
                    help="energy of an earlier run after --converge-iters iterations; dE of every mode against it")
    ap.add_argument("--batched-graph", type=int, default=1, help="1: replay a recorded graph, 0: enqueue eagerly")
    ap.add_argument("--batched-streams", type=int, default=4, help="streams the batch's systems are spread over")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (reference for the HBM byte counters)")
    ap.add_argument("--slab", action="store_true",
                    help="only the block-local terms of a 64-triple slab at o=50 v=400 (FP32 and split-BF16)")
    ap.add_argument("--panel", type=int, default=8, help="W rows a per rebuilt panel (--slab)")
    ap.add_argument("--q-workload", default="none", metavar="NAME",
                    help="also time the (Q) correction on this workload (e.g. o10v90-scaled)")
    ap.add_argument("--q-abc", action="store_true",
                    help="only the (Q) correction in the virtual-tuple order on sampled tasks of o20v180-weak")
    ap.add_argument("--q-abc-tasks", type=int, default=QABC["ntasks"])
    ap.add_argument("--q-abc-block", type=int, default=QABC["block"])
    ap.add_argument("--quad", action="store_true",
                    help="only the quadruples ladder on compact T4 (o=6 v=48), every mode")
    args = ap.parse_args(argv)
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

    if binding is None:
        from paper_2607_00981_amd import binding

    if args.q_abc:
        r = run_q_abc(binding, QABC["workload"], args.q_abc_block, args.q_abc_tasks)
        print(json.dumps({
            "metric": "(Q) correction, virtual-tuple order: matrix-core TFLOP/s over the sampled tasks, o=20 v=180",
            "value": r["tflops_mfma_over_tasks"], "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1000.0 * r["tasks_s"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic", "config": {"workload": r["workload"], "block": r["block"]},
            "q_abc": r,
            "roofline": {"bound": "mfma", "achieved": r["tflops_mfma_over_tasks"], "peak": r["peak"],
                         "unit": "TFLOP/s", "frac": r["frac"], "traffic": None,
                         "kernel": "all kernels of the sampled tasks (matrix-core products, gathers, Wbar builds, "
                                   "energy)"},
        }), flush=True)
        return

    if args.quad:
        modes = [args.precision] + [m for m in args.compare.split(",") if m and m != args.precision]
        res = run_quad(binding, modes)
        r = res["modes"][args.precision]
        print(json.dumps({
            "metric": "quadruples ladder TFLOP/s on compact T4 (RCCSDTQ), o=6 v=48",
            "value": r["tflops_wall"], "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": 1000.0 * r["s"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": DTYPE[args.precision], "data": "synthetic",
            "config": {"workload": res["workload"], "precision": args.precision},
            "modes": res["modes"],
            "roofline": {"bound": "mfma", "achieved": r["tflops_gemm"], "peak": r["peak"], "unit": "TFLOP/s",
                         "frac": r["frac_gemm"], "traffic": None,
                         "kernel": "ladder GEMMs batched over the stored blocks (six per evaluation)"},
        }), flush=True)
        return

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

    if args.converge:
        modes = [args.precision] + [m for m in args.compare.split(",") if m and m != args.precision]
        res = run_accuracy(binding, modes, tol=args.converge_tol, max_iter=args.converge_max_iter,
                           workload=args.converge, iters=args.converge_iters, ref_energy=args.converge_ref_energy)
        print(json.dumps({"converge": res, "wall_s": elapsed()}), flush=True)
        return

    budget_end = args.budget_s
    s = ci.make_named(args.workload)
    o, v, naux, seed = s["o"], s["v"], s["naux"], s["seed"]
    sigma = ci.variant_sigma(args.workload.partition("-")[2], naux)
    compare = [m for m in args.compare.split(",") if m and m != args.precision]
    samples = sample_offsets(o, v)
    log(f"[bench] {args.workload}: o={o} v={v} naux={naux} seed={seed} sigma={sigma:.6g} main={args.precision} "
        f"compare={compare} budget {args.budget_s:.0f} s")

    # the main mode's share of the budget: what the comparison modes, the
    # batch and the CPU baseline are estimated to need is kept back; the
    # estimate scales with the iteration time, known after the first one
    est_setup = 20.0
    est_cpu = 0.0 if args.no_cpu_baseline else args.cpu_seconds + 15.0
    est_batch = 45.0 if args.batched_iters > 1 else 0.0

    def main_end(t_it):
        return (budget_end - compare_reserve(compare, t_it, est_setup, 1 + max(args.compare_steps, 0))
                - est_cpu - est_batch - 5.0)

    skipped = []
    main_run = run_mode(binding, s, args.precision, args.steps, args.warmup, args.autotune_ms, samples, main_end)
    log(f"[bench] main mode done at t={elapsed():.0f} s")
    ms_step = main_run["ms_per_step"]
    t_it_main = ms_step / 1000.0
    value = 2.0 * main_run["r3_macs"] / (ms_step / 1000.0) / 1e12
    lad = main_run["ladder_gemm"]
    achieved = 2.0 * lad["macs"] / (lad["ms"] / 1000.0) / 1e12 if lad["ms"] > 0 else None
    peak = PEAK[args.precision]
    kname = kernel_name(args.precision, main_run["tile_variants"]["ladder"])
    traffic = stored_traffic(args.precision, args.workload, kname)
    e_main = main_run["energies"]
    modes = {args.precision: {"s_per_iteration": t_it_main, "r3_tflops": main_run["r3_tflops"],
                              "energies": e_main, "residual_norms": main_run["norms"], "speedup": 1.0,
                              "tile_variants": main_run["tile_variants"], "steps": main_run["steps"]}}
    for prec in compare:
        est = compare_reserve([prec], t_it_main, main_run["setup_s"], 1 + max(args.compare_steps, 0))
        if elapsed() + est > budget_end - est_cpu:
            skipped.append(f"mode {prec} (estimated {est:.0f} s, {budget_end - elapsed():.0f} s left)")
            log(f"[bench] skipping {prec}: estimate {est:.0f} s does not fit")
            continue
        try:
            r = run_mode(binding, s, prec, args.compare_steps, 1, args.autotune_ms, samples,
                         lambda _t: budget_end - est_cpu, main=False)
        except binding.CCTError as exc:
            modes[prec] = {"error": str(exc)}
            log(f"[bench] {prec} failed: {exc}")
            continue
        rec = {"s_per_iteration": r["ms_per_step"] / 1000.0, "r3_tflops": r["r3_tflops"], "energies": r["energies"],
               "residual_norms": r["norms"], "speedup": ms_step / r["ms_per_step"], "phase_ms": r["phase_ms"],
               "tile_variants": r["tile_variants"], "steps": r["steps"],
               "r3_rel_dev": r3_deviation(main_run["r3_samples"], r["r3_samples"])}
        n_cmp = min(len(e_main), len(r["energies"]))
        if n_cmp >= 1:
            dE = r["energies"][n_cmp - 1] - e_main[n_cmp - 1]
            rec.update({"dE": dE, "dE_rel": dE / max(abs(e_main[n_cmp - 1]), 1e-300), "dE_after_iterations": n_cmp})
        modes[prec] = rec
        log(f"[bench] {prec}: {r['ms_per_step'] / 1000:.2f} s/iteration, R3 deviation {rec['r3_rel_dev']}, "
            f"dE {rec.get('dE')}")
    out = {
        "metric": "T3-residual TFLOP/s + s/CCSDT iteration, FP64 vs mixed, o=20 v=180, dE vs oracle",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": main_run["steps"],
        "warmup": main_run["warmup"],
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"RCCSDT iteration o={o} v={v} naux={naux} seed={seed}, B entries N(0, {sigma:.6g}) "
                               f"({args.workload.partition('-')[2] or 'named'} recipe), compact T3 "
                               f"({o*(o+1)*(o+2)//6} triples x {v}^3), MP2 start, one untimed iteration, "
                               f"DIIS on T1/T2",
                   "precision": args.precision},
        "s_per_iteration": t_it_main,
        "step_s": main_run["step_s"],
        "r3_tflops": main_run["r3_tflops"],
        "value_direct_count": 2.0 * main_run["r3_macs_direct"] / (ms_step / 1000.0) / 1e12,
        "phase_ms": main_run["phase_ms"],
        "modes": modes,
        "modes_note": ("every mode starts from the same MP2 guess; after one iteration the state is identical in "
                       "every mode (T3 = 0 at the guess, so the mixed contractions contribute nothing in it); "
                       "r3_rel_dev = max|R3(mode) - R3(main)| / max|R3(main)| over the sampled packed blocks "
                       f"{[t for t, _, _ in samples]} of the residual of that state (iteration 2); dE = E(mode) - "
                       "E(main) after the same number of iterations (dE_after_iterations; the mixed contractions "
                       "reach the energy from iteration 3 on)"),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak if achieved else None, "traffic": traffic,
                     "traffic_source": ("profiles/pp_ladder_gemm_o20v180_fp64_traffic.md (FETCH_SIZE + WRITE_SIZE, "
                                        "copy-calibrated, stored; not measured by this run)") if traffic else None,
                     "kernel": kname + " (particle-particle ladder GEMMs)",
                     "launches_per_step": lad["launches"], "ms_per_launch": lad["ms"] / max(lad["launches"], 1),
                     "flop_per_launch": 2.0 * lad["macs"] / max(lad["launches"], 1)},
        "energy": main_run["energy"],
    }
    if args.batched_iters > 1:
        if elapsed() + est_batch > budget_end - est_cpu:
            skipped.append("batch leg")
        else:
            try:
                out["batched"] = run_batched(binding, args.batched_iters, [args.precision] + compare,
                                             args.autotune_ms, bool(args.batched_graph), args.batched_streams)
            except binding.CCTError as exc:
                out["batched"] = {"error": str(exc)}
    if args.accuracy:
        if elapsed() + 90.0 > budget_end - est_cpu:
            skipped.append("accuracy leg")
        else:
            out["accuracy"] = run_accuracy(binding, [args.precision] + compare)
    if args.q_workload and args.q_workload != "none":
        if elapsed() + 120.0 > budget_end - est_cpu:
            skipped.append("(Q) leg")
        else:
            log(f"[bench] (Q) correction on {args.q_workload} ...")
            out["q"] = run_q(binding, args.q_workload, cpu=not args.no_cpu_baseline)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(s, budget_s=args.cpu_seconds)
    out["skipped"] = skipped
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
