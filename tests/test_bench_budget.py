"""CPU: the benchmark's wall-budget logic.

bench.py is run in-process against a stand-in of the binding whose calls
advance a simulated clock by the measured per-call times of the o=20 v=180
workload on one MI355X (FP64 iteration ~30 s, FP32 ~21 s, split-BF16 ~10 s),
so the driver's request (--steps 20 --warmup 5) is replayed without a GPU:
the JSON line must come out, the simulated wall time must stay inside the
budget, the executed step counts must be the ones reported, and the mode
comparison must be taken on the iteration-2 residual of every mode.
"""

import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


class Clock:
    def __init__(self):
        self.t = 1000.0

    def __call__(self):
        return self.t


def fake_binding(clock, iter_s, setup_s=12.0, batch_s=6.0):
    """A stand-in of paper_2607_00981_amd.binding: every call advances the
    clock; update() returns a fixed energy trajectory per mode."""

    class CCTError(RuntimeError):
        pass

    PHASES = ("ccsd", "feedback", "pp", "rings", "hh_f2", "drivers", "f1", "post", "diis_energy")
    TERMS = {"D1": 1, "D2": 2, "F1": 4, "F2": 8, "RA": 16, "RB": 32, "RC": 64, "HH": 128, "PP": 256}
    calls = {"update": {}, "copy_r3": {}}

    class Engine:
        def __init__(self, o, v, naux, precision="fp64", opts=None):
            self.prec = precision
            self.it = 0
            clock.t += setup_s / 2

        def set_fock(self, f):
            pass

        def set_eri_df(self, B):
            clock.t += 1.0

        def init_mp2(self):
            pass

        def autotune(self, ms):
            clock.t += ms / 1000.0 + setup_s / 2
            return (1, 1)

        def update(self):
            clock.t += iter_s[self.prec]
            self.it += 1
            calls["update"][self.prec] = calls["update"].get(self.prec, 0) + 1
            # identical energies for the first two iterations, then a mode shift
            e = -10.0 - 0.1 * self.it + (1e-9 * {"fp64": 0, "fp32": 1, "bf16x3": 5}[self.prec] if self.it >= 3 else 0)
            return e, np.array([1e-4, 1e-4, 1e-4]) / self.it

        def counters(self):
            macs = {k: 1e12 for k in TERMS}
            macs["ladder_gemm"], macs["ladder_launches"] = 4.4e14, 12.0
            ms = {k: 1000.0 * iter_s[self.prec] / 10 for k in PHASES}
            ms["ladder_gemm"] = 1000.0 * iter_s[self.prec] * 0.45
            return macs, ms

        def copy_r3(self, first, count):
            calls["copy_r3"].setdefault(self.prec, []).append(self.it)
            base = np.linspace(-1.0, 1.0, 16)
            return base * (1.0 + {"fp64": 0.0, "fp32": 1e-7, "bf16x3": 1e-5}[self.prec])

        def close(self):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

    class Batch:
        def __init__(self, sizes, precision="fp64", opts=None):
            self.n = len(sizes)

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

        def set_system(self, k, f, B):
            pass

        def autotune(self, ms):
            clock.t += ms / 1000.0

        def iterate(self, n):
            clock.t += batch_s / 5 * n
            return np.full(self.n, -1.0), np.zeros((self.n, 3))

    ns = type("binding", (), {})()
    ns.Engine, ns.Batch, ns.CCTError, ns.PHASES, ns.TERMS, ns.calls = Engine, Batch, CCTError, PHASES, TERMS, calls
    return ns


@pytest.fixture
def sim(monkeypatch):
    clock = Clock()
    monkeypatch.setattr(bench, "_now", clock)
    monkeypatch.setattr(bench, "T_START", clock.t)

    def fake_cpu(s, budget_s=10.0, max_blocks=12):
        clock.t += budget_s + 8.0
        return {"value": 0.3, "unit": "TFLOP/s", "cores": 16, "kind": "oracle", "sample": "simulated"}

    monkeypatch.setattr(bench, "cpu_baseline", fake_cpu)
    return clock


ITER_S = {"fp64": 30.0, "fp32": 21.0, "bf16x3": 10.0}


def _run(capsys, clock, argv, iter_s=ITER_S):
    b = fake_binding(clock, iter_s)
    bench.main(argv, binding=b)
    lines = [ln for ln in capsys.readouterr().out.splitlines() if ln.strip()]
    assert len(lines) == 1
    return json.loads(lines[0]), b, clock.t - bench.T_START


def test_plan_steps():
    assert bench.plan_steps(20, 30.0, 160.0) == 5
    assert bench.plan_steps(20, 30.0, 10.0) == 1       # at least one timed step
    assert bench.plan_steps(3, 30.0, 1000.0) == 3      # never more than requested
    assert bench.plan_steps(0, 30.0, 1000.0) == 0
    assert bench.plan_extra_warmup(4, 30.0, 65.0) == 2
    assert bench.plan_extra_warmup(4, 30.0, -5.0) == 0
    assert bench.compare_reserve(["fp32", "bf16x3"], 30.0, 10.0, 3) == pytest.approx(10 + 67.5 + 10 + 36)


def test_driver_request_fits_budget(sim, capsys):
    d, b, wall = _run(capsys, sim, ["--steps", "20", "--warmup", "5"])
    assert wall <= 450.0
    assert 1 <= d["steps"] < 20 and d["steps_requested"] == 20 and d["warmup_requested"] == 5
    assert b.calls["update"]["fp64"] == d["steps"] + d["warmup"]
    assert d["ms_per_step"] * d["steps"] / 1000.0 < wall
    assert d["config"]["workload"].startswith("RCCSDT iteration o=20 v=180 naux=400 seed=3")
    assert d["dtype"] == "f64" and d["roofline"]["bound"] == "mfma" and d["cpu_baseline"]["kind"] == "oracle"
    # both comparison modes ran, their R3 samples come from iteration 2 like the main mode's
    assert set(d["modes"]) == {"fp64", "fp32", "bf16x3"}
    for m in ("fp64", "fp32", "bf16x3"):
        assert set(b.calls["copy_r3"][m]) == {2}
    assert d["modes"]["bf16x3"]["r3_rel_dev"] == pytest.approx(1e-5)
    assert d["modes"]["fp32"]["r3_rel_dev"] == pytest.approx(1e-7)
    assert d["modes"]["bf16x3"]["dE_after_iterations"] == 3
    assert d["modes"]["bf16x3"]["dE"] == pytest.approx(5e-9, abs=1e-12)


def test_slow_machine_still_prints(sim, capsys):
    slow = {k: 3 * x for k, x in ITER_S.items()}
    d, b, wall = _run(capsys, sim, ["--steps", "20", "--warmup", "5"], iter_s=slow)
    # one warm-up and one timed step always run; what does not fit is skipped and named
    assert d["steps"] >= 1 and d["warmup"] >= 1
    assert d["skipped"]
    assert wall <= 450.0 + 3 * 30.0


def test_small_request_runs_exactly(sim, capsys):
    d, b, wall = _run(capsys, sim, ["--steps", "2", "--warmup", "1", "--compare", "bf16x3"])
    assert d["steps"] == 2 and d["warmup"] == 1
    assert b.calls["update"]["fp64"] == 3
    assert set(d["modes"]) == {"fp64", "bf16x3"} and not d["skipped"]


def test_converge_leg_stops_at_tolerance_and_matches_iterations(sim, capsys):
    # the fake squared norms sum to 3e-4 / iteration: |R| < 7e-3 from iteration 7 on
    d, b, _ = _run(capsys, sim, ["--converge", "o4v20-weak", "--converge-tol", "7e-3", "--compare", "bf16x3"])
    c = d["converge"]
    assert c["fp64"]["iterations"] == 7 and c["bf16x3"]["iterations"] == 7
    assert len(c["fp64"]["energies"]) == 7 and c["fp64"]["residual_norms"][-1] < 7e-3
    assert c["bf16x3"]["dE"] == pytest.approx(5e-9, abs=1e-12)
    assert "o=4 v=20 naux=48" in c["workload"]


def test_converge_leg_against_a_stored_reference_energy(sim, capsys):
    d, b, _ = _run(capsys, sim, ["--converge", "o4v20-weak", "--precision", "bf16x3", "--compare", "fp32",
                                 "--converge-iters", "4", "--converge-ref-energy", "-10.4"])
    c = d["converge"]
    assert b.calls["update"] == {"bf16x3": 4, "fp32": 4}
    assert c["bf16x3"]["dE"] == pytest.approx(5e-9, abs=1e-12)
    assert c["fp32"]["dE"] == pytest.approx(1e-9, abs=1e-12)
