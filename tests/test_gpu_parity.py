"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Inputs come from cct_inputs (seeded); expected values from oracle/ only.
Tolerances: FP64 residuals agree to 1e-11 relative to the largest residual
element (roundoff of a few-thousand-term sums is ~1e-14 relative); energies
after 20 iterations to 1e-10 Eh.  Mixed modes (ladder and ring contractions
on FP32 or split-BF16 operands, FP32 accumulation over 128 products):
operand rounding is 2^-24 (FP32) or about 2^-17 (hi+lo BF16) relative, so
R3 is held to 2e-6 (FP32) and 5e-5 (BF16X3) of its largest element, and the
energy after 20 DIIS iterations to 1e-6 Eh of the FP64 oracle.
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


def _system(o, v, seed, sigma=0.1, nondiag=True):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=sigma)
    f = ci.random_fock(o, v, seed) if nondiag else s["f"]
    return f, s["B"]


def _amps(o, v, seed, s3=0.02):
    t1, t2, _ = ci.random_amplitudes(o, v, seed, 0.02, 0.03, 0.0, triples=False)
    t3p = ci.random_t3_packed(o, v, seed + 100, s3)
    return t1, t2, t3p


def _engine(o, v, naux, f, B, **kw):
    eng = binding.Engine(o, v, naux, **kw)
    eng.set_fock(f)
    eng.set_eri_df(B)
    return eng


def _oracle_residual(f, B, o, t1, t2, t3p, terms=None):
    V = R.eri_phys_from_B(B)
    t3 = R.unpack_t3(t3p, o)
    r1, r2, r3 = R.residuals(f, V, t1, t2, t3, o, terms=terms)
    return r1, r2, R.pack_t3(R.postprocess_r3(r3))


def _close(a, b, rel=1e-11):
    scale = max(1.0, float(np.abs(b).max()))
    err = float(np.abs(a - b).max())
    return err <= rel * scale, err, scale


@pytest.mark.parametrize("shape", [(3, 7, 31), (3, 8, 32)], ids=["odd_v", "even_v"])
@pytest.mark.parametrize("term", R.R3_TERMS)
def test_each_r3_term_matches_oracle(term, shape):
    """Each term group alone; odd v runs the generic strided kernels, even v
    the K-contiguous matrix-core path."""
    o, v, seed = shape
    say(f"[term parity] term={term} o={o} v={v} seed={seed}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    e1, e2, e3 = _oracle_residual(f, B, o, t1, t2, t3p, terms=(term,))
    with _engine(o, v, B.shape[0], f, B) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        g1, g2, g3, _ = eng.residual([term])
    for name, a, b in (("R1", g1, e1), ("R2", g2, e2), ("R3", g3, e3)):
        ok, err, scale = _close(a, b)
        assert ok, f"{name} term {term}: max err {err:.3e} (scale {scale:.3e})"
    assert np.abs(e3).max() > 1e-6


@pytest.mark.parametrize("o,v,seed", [(1, 5, 3), (2, 3, 4), (3, 9, 5), (4, 20, 6), (5, 11, 7)])
def test_full_residual_matches_oracle(o, v, seed):
    say(f"[full parity] o={o} v={v} seed={seed}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    e1, e2, e3 = _oracle_residual(f, B, o, t1, t2, t3p)
    with _engine(o, v, B.shape[0], f, B) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        g1, g2, g3, nr = eng.residual()
    for name, a, b in (("R1", g1, e1), ("R2", g2, e2), ("R3", g3, e3)):
        ok, err, scale = _close(a, b)
        assert ok, f"{name}: max err {err:.3e} (scale {scale:.3e})"
    w = np.array([R.multiplicity(*t) for t in R.packed_list(o)], dtype=float)
    n3 = float(np.sum(w[:, None, None, None] * e3 * e3))
    assert abs(nr[2] - n3) <= 1e-10 * max(1.0, n3)
    assert abs(nr[0] - np.sum(e1 * e1)) <= 1e-10 * max(1.0, np.sum(e1 * e1))


def test_mp2_guess_energy_anchor():
    o, v, naux, seed = ci.CONFIGS["o4v20"]
    say("[mp2 anchor]")
    s = ci.make_system(o, v, naux, seed)
    with _engine(o, v, naux, s["f"], s["B"]) as eng:
        eng.init_mp2()
        e = eng.energy()
    V = R.eri_phys_from_B(s["B"])
    t1, t2, _ = R.mp2_guess(s["f"], V, o)
    assert abs(e - R.energy(s["f"], V, t1, t2, o)) < 1e-12


def test_residual_is_bitwise_deterministic():
    o, v, seed = 4, 13, 9
    say("[determinism]")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    with _engine(o, v, B.shape[0], f, B) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        a = eng.residual()
        b = eng.residual()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("diis", [True, False])
def test_twenty_iterations_o4v20(diis):
    """Twenty iterations from the MP2 guess on the o=4, v=20 workload (seed 1):
    GPU energy after every iteration within 1e-10 Eh of the oracle."""
    o, v, naux, seed = ci.CONFIGS["o4v20"]
    niter = 20 if diis else 8
    say(f"[iterations] diis={diis} niter={niter}")
    s = ci.make_system(o, v, naux, seed)
    f, B = s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS() if diis else None
    ref = []
    for _ in range(niter):
        t1, t2, t3, e, _ = R.iterate(f, V, t1, t2, t3, o, diis=d)
        ref.append(e)
    opts = {"diis": diis}
    with _engine(o, v, naux, f, B, opts=opts) as eng:
        eng.init_mp2()
        got = []
        for it in range(niter):
            e, nr = eng.update()
            got.append(e)
            say(f"  it {it+1}: gpu {e:.14f} oracle {ref[it]:.14f} diff {e-ref[it]:.2e}")
        g1, g2, g3 = eng.get_amplitudes()
    assert np.max(np.abs(np.array(got) - np.array(ref))) < 1e-10
    assert np.abs(g3 - R.pack_t3(t3)).max() < 1e-9


MIXED_TOL = {"fp32": 2e-6, "bf16x3": 5e-5}


@pytest.mark.parametrize("shape", [(3, 7, 31), (3, 8, 32), (2, 12, 41)], ids=["odd_v", "even_v", "v12"])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_residual_close_to_oracle(prec, shape):
    """v=8 and v=12 take the low-precision operand kernels (K multiple of the
    vector width), v=7 the generic strided kernels with operands rounded at
    the LDS store.  R1 and R2 stay FP64."""
    o, v, seed = shape
    say(f"[mixed parity] prec={prec} o={o} v={v} seed={seed}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    e1, e2, e3 = _oracle_residual(f, B, o, t1, t2, t3p)
    with _engine(o, v, B.shape[0], f, B, precision=prec) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        g1, g2, g3, _ = eng.residual()
    for name, a, b, rel in (("R1", g1, e1, 1e-11), ("R2", g2, e2, 1e-11), ("R3", g3, e3, MIXED_TOL[prec])):
        ok, err, scale = _close(a, b, rel)
        say(f"  {name}: max err {err:.3e} scale {scale:.3e}")
        assert ok, f"{prec} {name}: max err {err:.3e} (scale {scale:.3e})"
    # the rounding is really there: FP32/BF16 operands do not reproduce FP64 bit for bit
    assert not np.array_equal(g3, e3)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_twenty_iterations_o4v20(prec):
    """Twenty DIIS iterations from the MP2 guess at o=4, v=20 in a mixed mode:
    the energy stays within 1e-6 Eh of the FP64 oracle at every iteration."""
    o, v, naux, seed = ci.CONFIGS["o4v20"]
    say(f"[mixed iterations] prec={prec}")
    s = ci.make_system(o, v, naux, seed)
    f, B = s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS()
    ref = []
    for _ in range(20):
        t1, t2, t3, e, _ = R.iterate(f, V, t1, t2, t3, o, diis=d)
        ref.append(e)
    with _engine(o, v, naux, f, B, precision=prec) as eng:
        eng.init_mp2()
        got = []
        for it in range(20):
            e, nr = eng.update()
            got.append(e)
            say(f"  it {it+1}: gpu {e:.14f} oracle {ref[it]:.14f} diff {e-ref[it]:.2e}")
    assert np.max(np.abs(np.array(got) - np.array(ref))) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_autotune_keeps_results_and_writes_cache(prec, tmp_path, monkeypatch):
    """Tuned tile variants give the untuned residual to rounding, the choice
    lands in the cache file, and a new context picks it up from there."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("CCT_TUNE_CACHE", str(cache))
    o, v, seed = 3, 16, 21
    say(f"[autotune] prec={prec}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    with _engine(o, v, B.shape[0], f, B, precision=prec) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        a = eng.residual()
        lad, rng = eng.autotune(500.0)
        say(f"  variants ladder={lad} rings={rng}")
        b = eng.residual()
    for x, y in zip(a[:3], b[:3]):
        assert np.abs(x - y).max() <= 1e-12 * max(1.0, np.abs(x).max())
    import json
    js = json.loads(cache.read_text())
    assert js[f"o{o}_v{v}_{prec}_ladder_split"] == lad and js[f"o{o}_v{v}_{prec}_rings"] == rng
    with _engine(o, v, B.shape[0], f, B, precision=prec) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        c = eng.residual()
    for x, y in zip(b[:3], c[:3]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("shape", [(3, 7, 31), (3, 8, 32)], ids=["odd_v", "even_v"])
def test_direct_ladder_matches_oracle(shape):
    """The direct-traversal ladder (symmetric/antisymmetric split switched
    off) against the oracle's PP term."""
    o, v, seed = shape
    say(f"[direct ladder] o={o} v={v} seed={seed}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    _, _, e3 = _oracle_residual(f, B, o, t1, t2, t3p, terms=("PP",))
    with _engine(o, v, B.shape[0], f, B, opts={"ladder_split": False}) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        _, _, g3, _ = eng.residual(["PP"])
    ok, err, scale = _close(g3, e3)
    assert ok, f"direct ladder: max err {err:.3e} (scale {scale:.3e})"


# (o, v, workspace cap in GB): v = 2 (one pair tile, padding of K), v = 33
# (ragged second pair tile), v = 70 (three tiles); the last case caps the
# workspace so that the 56 packed blocks are split over two chunks.
SPLIT_CASES = [(2, 2, 0.0), (3, 33, 0.0), (2, 70, 0.0), (6, 60, 0.001)]


@pytest.mark.parametrize("o,v,ws", SPLIT_CASES, ids=["v2", "v33", "v70", "v60_chunks"])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_ladder_split_matches_direct(prec, o, v, ws):
    """The symmetric/antisymmetric ladder against the direct traversal in
    FP64 (PP term alone, same inputs): FP64 agrees to summation order, the
    mixed modes to their operand rounding.  The executed multiply-adds are
    v(v+1)/2 v^2 per row and term against v^4 for the direct form."""
    seed = 40 + v
    say(f"[ladder split] prec={prec} o={o} v={v} ws={ws}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    opts = {"timers": True}
    if ws:
        opts["workspace_gb"] = ws
    with _engine(o, v, B.shape[0], f, B, opts=dict(opts, ladder_split=False)) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        _, _, ref, _ = eng.residual(["PP"])
    with _engine(o, v, B.shape[0], f, B, precision=prec, opts=opts) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        _, _, got, _ = eng.residual(["PP"])
        macs, _ = eng.counters()
    rel = 1e-12 if prec == "fp64" else MIXED_TOL[prec]
    ok, err, scale = _close(got, ref, rel)
    say(f"  max err {err:.3e} scale {scale:.3e}")
    assert ok, f"split ladder {prec}: max err {err:.3e} (scale {scale:.3e})"
    assert np.abs(ref).max() > 1e-6
    ntri = o * (o + 1) * (o + 2) // 6
    assert macs["ladder_gemm"] == 3 * ntri * v * (v * (v + 1) // 2) * v * v
    assert macs["PP"] == 3 * ntri * v ** 5


TILE_VARIANTS = {"fp64": (1, 2, 3, 4, 9, 10, 11), "fp32": (1, 2, 3, 5), "bf16x3": (1, 2, 3, 4, 5)}
CASES = [(p, x, False) for p, vs in TILE_VARIANTS.items() for x in vs] + [("bf16x3", x, True) for x in (1, 2, 3, 4, 5)]


@pytest.mark.parametrize("prec,var,blocked", CASES)
def test_every_tile_variant_matches_oracle(prec, var, blocked, tmp_path, monkeypatch):
    """Each GEMM tile variant, forced for the ladder and the rings through the
    tuning cache, on a shape whose GEMMs all end in ragged tiles (v = 30:
    465 pairs, o v = 90, 10 packed blocks).  blocked: the split-BF16 ladder
    and ring operands in the layout interleaved by blocks of 32 (forced at
    this size through lp_block_k = 0; K padded to 480, 448 and 96)."""
    import json

    o, v, seed = 3, 30, 23
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({f"o{o}_v{v}_{prec}_ladder_split": var, f"o{o}_v{v}_{prec}_rings": var}))
    monkeypatch.setenv("CCT_TUNE_CACHE", str(cache))
    say(f"[tile variant] prec={prec} variant={var} blocked={blocked}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    e1, e2, e3 = _oracle_residual(f, B, o, t1, t2, t3p)
    opts = {"lp_block_k": 0} if blocked else None
    with _engine(o, v, B.shape[0], f, B, precision=prec, opts=opts) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        g1, g2, g3, _ = eng.residual()
    rel = 1e-11 if prec == "fp64" else MIXED_TOL[prec]
    for name, a, b, r in (("R1", g1, e1, 1e-11), ("R2", g2, e2, 1e-11), ("R3", g3, e3, rel)):
        ok, err, scale = _close(a, b, r)
        say(f"  {name}: max err {err:.3e} scale {scale:.3e}")
        assert ok, f"{prec} variant {var} {name}: max err {err:.3e} (scale {scale:.3e})"


@pytest.mark.parametrize("o,v", [(3, 33), (4, 20)])
def test_blocked_split_bf16_layout_is_a_storage_layout_only(o, v):
    """The split-BF16 residual with the ladder and ring operands interleaved
    by blocks of 32 (lp_block_k = 0) equals the one with two planes
    (lp_block_k above every K) element for element: both feed the same
    products to the same accumulators in the same K order; only the zero
    padding of K differs (8 against 32), and adding exact zeros changes no
    FP32 sum.  v = 33: ragged pair tiles, K = 561 / 528 pairs; o v = 99 and
    80 ring columns."""
    seed = 70 + v
    say(f"[blocked layout] o={o} v={v}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    out = []
    for k in (0, 1 << 40):
        with _engine(o, v, B.shape[0], f, B, precision="bf16x3", opts={"lp_block_k": k}) as eng:
            eng.set_amplitudes(t1, t2, t3p)
            out.append(eng.residual())
    for name, a, b in zip(("R1", "R2", "R3"), out[0][:3], out[1][:3]):
        d = float(np.abs(a - b).max())
        say(f"  {name}: max |blocked - planar| {d:.3e}")
        assert np.array_equal(a, b), f"{name} differs by {d:.3e}"
    assert np.abs(out[0][2]).max() > 1e-6


@pytest.mark.parametrize("mode", ["subspace:10", "none"])
def test_twenty_iterations_partial_t3_diis(mode):
    """DIIS with T3 restricted to the first 10 virtuals (or left out): the
    GPU energies follow the oracle run with the same reading to 1e-10 Eh per
    iteration, and the run differs from whole-T3 DIIS (the option acts)."""
    o, v, naux, seed = ci.CONFIGS["o4v20"]
    niter = 20
    say(f"[partial T3 DIIS] mode={mode}")
    s = ci.make_system(o, v, naux, seed)
    f, B = s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    omode = "none" if mode == "none" else int(mode.split(":")[1])
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS()
    ref = []
    for _ in range(niter):
        t1, t2, t3, e, _ = R.iterate(f, V, t1, t2, t3, o, diis=d, diis_t3=omode)
        ref.append(e)
    got = {}
    for m in (mode, "full"):
        with _engine(o, v, naux, f, B, opts={"diis_t3": m}) as eng:
            eng.init_mp2()
            got[m] = [eng.update()[0] for _ in range(niter)]
            if m == mode:
                g1, g2, g3 = eng.get_amplitudes()
    for it in range(niter):
        say(f"  it {it+1}: gpu {got[mode][it]:.14f} oracle {ref[it]:.14f} diff {got[mode][it]-ref[it]:.2e}")
    assert np.max(np.abs(np.array(got[mode]) - np.array(ref))) < 1e-10
    assert np.abs(g3 - R.pack_t3(t3)).max() < 1e-9
    assert np.max(np.abs(np.array(got[mode]) - np.array(got["full"]))) > 1e-12


def test_solve_takes_the_tol_option():
    """cct_solve with tol <= 0 stops at the context's "tol" option; a tighter
    explicit threshold needs more iterations and lands on the oracle's
    converged energy."""
    o, v, seed = 2, 8, 61
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=0.1)
    f, B = s["f"], s["B"]
    say("[solve tol]")
    with _engine(o, v, B.shape[0], f, B, opts={"tol": 1e-5}) as eng:
        eng.init_mp2()
        e1, it1, ok1 = eng.solve(200)
    with _engine(o, v, B.shape[0], f, B) as eng:
        eng.init_mp2()
        e2, it2, ok2 = eng.solve(200, tol=1e-11)
    assert ok1 and ok2 and it2 > it1
    eref, *_, conv = R.solve(f, R.eri_phys_from_B(B), o, tol=1e-11, max_iter=200)
    assert conv and abs(e2 - eref) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
@pytest.mark.parametrize("o,v", [(1, 1), (2, 1), (1, 2), (3, 2), (2, 3)])
def test_degenerate_shapes_match_oracle(prec, o, v):
    """Smallest shapes: a single virtual (no virtual pairs off the diagonal,
    the ladder falls back to the direct form), a single occupied (one packed
    block, i=j=k), two virtuals (one pair tile, K padded far beyond v(v+1)/2)."""
    seed = 70 + 10 * o + v
    say(f"[degenerate] prec={prec} o={o} v={v}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    e1, e2, e3 = _oracle_residual(f, B, o, t1, t2, t3p)
    with _engine(o, v, B.shape[0], f, B, precision=prec) as eng:
        eng.set_amplitudes(t1, t2, t3p)
        g1, g2, g3, _ = eng.residual()
    rel = 1e-11 if prec == "fp64" else MIXED_TOL[prec]
    for name, a, b, r in (("R1", g1, e1, 1e-11), ("R2", g2, e2, 1e-11), ("R3", g3, e3, rel)):
        ok, err, scale = _close(a, b, r)
        assert ok, f"{prec} o={o} v={v} {name}: max err {err:.3e} (scale {scale:.3e})"


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_all_terms_with_every_job_in_several_batches(prec):
    """The whole residual with the workspace at its minimum (workspace_gb
    capped far below need), so that the T3 feedback, the three ring types,
    the hole ladder and both T2 drivers each run in two or more batches of
    unpacked slabs (slot offsets and per-batch fold plans of the multi-batch
    path the o=20 v=180 workload takes), against the oracle."""
    o, v, seed = 6, 24, 61
    say(f"[multi-batch] prec={prec} o={o} v={v}")
    f, B = _system(o, v, seed)
    t1, t2, t3p = _amps(o, v, seed)
    e1, e2, e3 = _oracle_residual(f, B, o, t1, t2, t3p)
    with _engine(o, v, B.shape[0], f, B, precision=prec, opts={"workspace_gb": 0.001}) as eng:
        plan = eng.batch_plan()
        say(f"  batch plan {plan}")
        for job in ("feedback", "ring_a", "ring_b", "ring_c", "hh", "d1", "d2"):
            assert plan[job] >= 2, (job, plan)
        eng.set_amplitudes(t1, t2, t3p)
        g1, g2, g3, _ = eng.residual()
    rel3 = 1e-11 if prec == "fp64" else MIXED_TOL[prec]
    for name, a, b, rel in (("R1", g1, e1, 1e-11), ("R2", g2, e2, 1e-11), ("R3", g3, e3, rel3)):
        ok, err, scale = _close(a, b, rel)
        say(f"  {name}: max err {err:.3e} scale {scale:.3e}")
        assert ok, f"{name} {prec}: max err {err:.3e} (scale {scale:.3e})"
