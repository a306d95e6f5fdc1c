"""Batches of independent systems through the C ABI (cct_batch_*).

Checks: (1) graph replay against eager enqueueing of the same batch and
against separate single-system contexts, iteration by iteration, bit for bit
(the same kernels run in the same order on the same data); (2) every system
against the FP64 oracle after each iteration (1e-10 Eh); (3) mixed-precision
batches within 1 microhartree of the FP64 batch.  Each replay is a separate
cct_batch_iterate call, so eager host work (DIIS, energies, read-backs)
and synchronisations run between replays.
"""

import sys

import numpy as np
import pytest

import cct_inputs as ci
from oracle import rccsdt as R
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu

SMALL = [(1, 6, 14, 11), (2, 7, 18, 12), (3, 9, 24, 13), (2, 12, 28, 14), (4, 10, 28, 15), (3, 16, 38, 16)]
NIT = 6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _systems(sizes):
    return [ci.make_system(o, v, na, seed) for o, v, na, seed in sizes]


def _batch_energies(sizes, systems, precision="fp64", graph=True, niter=NIT):
    out = []
    with binding.Batch([(o, v, na) for o, v, na, _ in sizes], precision=precision,
                       opts={"graph": graph}) as b:
        for k, s in enumerate(systems):
            b.set_system(k, s["f"], s["B"])
        for _ in range(niter):
            e, nr = b.iterate(1)
            assert np.all(np.isfinite(nr))
            out.append(e.copy())
    return np.array(out)  # [iteration][system]


def test_batch_graph_eager_single_and_oracle():
    systems = _systems(SMALL)
    say("[batch] graph replay")
    eg = _batch_energies(SMALL, systems, graph=True)
    say("[batch] eager")
    ee = _batch_energies(SMALL, systems, graph=False)
    assert np.array_equal(eg, ee)
    for k, (o, v, na, seed) in enumerate(SMALL):
        s = systems[k]
        with binding.Engine(o, v, na) as eng:
            eng.set_fock(s["f"])
            eng.set_eri_df(s["B"])
            eng.init_mp2()
            single = [eng.update()[0] for _ in range(NIT)]
        assert np.array_equal(np.array(single), eg[:, k]), f"system {k}"
        V = R.eri_phys_from_B(s["B"])
        t1, t2, t3 = R.mp2_guess(s["f"], V, o)
        d = R.DIIS()
        ref = []
        for _ in range(NIT):
            t1, t2, t3, e, _ = R.iterate(s["f"], V, t1, t2, t3, o, diis=d)
            ref.append(e)
        err = np.abs(eg[:, k] - np.array(ref)).max()
        say(f"  system {k} o={o} v={v}: E={eg[-1, k]:.12f} max |dE| vs oracle {err:.2e}")
        assert err < 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batch_mixed_close_to_fp64(prec):
    systems = _systems(SMALL)
    ref = _batch_energies(SMALL, systems)
    got = _batch_energies(SMALL, systems, precision=prec)
    d = np.abs(got - ref).max()
    say(f"[batch {prec}] max |dE| vs fp64 over {NIT} iterations: {d:.3e}")
    assert d < 1e-6


def test_batch_autotune_then_graph_matches_eager():
    """After tuning, the re-recorded graph still reproduces eager enqueueing."""
    systems = _systems(SMALL)
    ref = _batch_energies(SMALL, systems, graph=False)
    out = []
    with binding.Batch([(o, v, na) for o, v, na, _ in SMALL], opts={"graph": True}) as b:
        for k, s in enumerate(systems):
            b.set_system(k, s["f"], s["B"])
        b.iterate(1)
        out.append(None)
        b.autotune(200.0)
        for _ in range(NIT - 1):
            e, _ = b.iterate(1)
            out.append(e.copy())
    got = np.array(out[1:])
    assert np.abs(got - ref[1:]).max() < 1e-12
