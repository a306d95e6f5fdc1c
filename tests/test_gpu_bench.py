"""GPU: the benchmark's output contract on a small workload.

bench.py prints exactly one JSON line with the metric, the rate, the timing
fields, the roofline object of the dominant kernel and the CPU-oracle
baseline; a request for more than one GPU is refused with a message.
"""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, timeout=240):
    print(f"[bench contract] bench.py {' '.join(args)}", flush=True)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT, capture_output=True,
                          text=True, timeout=timeout)


def test_bench_prints_one_complete_json_line():
    p = _bench("--workload", "o4v20", "--steps", "2", "--warmup", "1", "--compare", "bf16x3", "--batched-iters", "2",
               "--autotune-ms", "100", "--q-workload", "none")
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, p.stdout
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["data"] == "synthetic"
    assert "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] > 0 and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]
    assert set(d["modes"]) == {"fp64", "bf16x3"} and not d["skipped"]
    m = d["modes"]["bf16x3"]
    # the mode comparison is taken on the same state (iteration-2 residual)
    assert 0.0 < m["r3_rel_dev"] < 5e-5 and m["dE_after_iterations"] == 3 and abs(m["dE"]) < 1e-6
    assert d["modes"]["fp64"]["energies"][0] == m["energies"][0]
    assert set(d["batched"]["modes"]) == {"fp64", "bf16x3"}


def test_bench_q_leg():
    p = _bench("--workload", "o4v20", "--steps", "1", "--warmup", "0", "--compare", "", "--batched-iters", "0",
               "--no-cpu-baseline", "--autotune-ms", "0", "--q-workload", "o4v20")
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, p.stdout
    q = json.loads(lines[0])["q"]
    assert q["workload"] == "o4v20" and q["s"] > 0 and q["algorithmic_flop"] > 0
    assert q["e_q"] != 0.0 and abs(q["frac"] - q["tflops"] / q["peak"]) < 1e-12


def test_bench_refuses_more_than_one_gpu():
    p = _bench("--gpus", "2", timeout=60)
    assert p.returncode != 0
    assert "one GPU" in p.stdout
