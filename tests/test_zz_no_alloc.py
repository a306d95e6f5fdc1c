"""GPU: the no-allocation (Q) entry point (cct_energy_q_noalloc) against the
allocating one (cct_energy_q), through the C ABI.

Two calls in a row on one GPU, the second with a smaller system (o=4 v=20,
then o=3 v=12), each compared with cct_energy_q on the same context: the
same kernels run in the same order, so the energies and per-task
contributions agree bit for bit (the second call runs on scratch that still
holds the first call's data).  The contexts use a counting caller allocator:
cct_energy_q takes blocks from it, cct_energy_q_noalloc none.  A system
whose buffers exceed the fixed scratch is refused with CCT_ENOMEM.
"""

import ctypes as C
import sys

import numpy as np
import pytest

import cct_inputs as ci
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class CountingAllocator:
    """hipMalloc / hipFree of the runtime libcct uses, counting calls."""

    def __init__(self):
        binding.load()
        with open("/proc/self/maps") as f:
            paths = {line.split()[-1] for line in f if "libamdhip64" in line}
        assert paths, "libamdhip64 is not loaded"
        self.hip = C.CDLL(sorted(paths)[0])
        self.hip.hipMalloc.restype = C.c_int
        self.hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.hip.hipFree.restype = C.c_int
        self.hip.hipFree.argtypes = [C.c_void_p]
        self.calls = 0
        self.live = set()

    def alloc(self, nbytes):
        self.calls += 1
        p = C.c_void_p()
        if self.hip.hipMalloc(C.byref(p), nbytes) != 0:
            return None
        self.live.add(p.value)
        return p.value

    def free(self, ptr):
        self.live.discard(ptr)
        self.hip.hipFree(C.c_void_p(ptr))

    def pair(self):
        return self.alloc, self.free


def _state(o, v, seed):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=ci.scaled_sigma(2 * (o + v)))
    t1, t2, _ = ci.random_amplitudes(o, v, seed, 0.0, 0.03, 0.0, triples=False)
    t3p = ci.random_t3_packed(o, v, seed + 1, 0.02)
    return s, t1, t2, t3p


def test_energy_q_noalloc_matches_energy_q():
    alloc = CountingAllocator()
    for o, v, seed in ((4, 20, 71), (3, 12, 72)):
        say(f"[noalloc] (Q) o={o} v={v} seed={seed}")
        s, t1, t2, t3p = _state(o, v, seed)
        with binding.Engine(o, v, s["naux"], allocator=alloc.pair()) as eng:
            eng.set_fock(s["f"])
            eng.set_eri_df(s["B"])
            eng.set_amplitudes(t1, t2, t3p)
            calls = alloc.calls
            e0, t0 = eng.energy_q_noalloc(tasks=True)
            assert alloc.calls == calls, "the no-allocation entry point allocated"
            e1, t1_ = eng.energy_q(tasks=True)
            assert alloc.calls > calls
            calls = alloc.calls
            e2, t2_ = eng.energy_q_noalloc(tasks=True)
            assert alloc.calls == calls
        say(f"  E_(Q) noalloc {e0:.15e} allocating {e1:.15e} noalloc again {e2:.15e}")
        assert e0 != 0.0
        assert abs(e0 - e1) <= 1e-11 * abs(e1) and e0 == e1 and e2 == e1
        assert np.array_equal(t0, t1_) and np.array_equal(t2_, t1_)
    assert not alloc.live


def test_energy_q_noalloc_refuses_systems_beyond_the_scratch():
    o, v, seed = 6, 24, 73
    say(f"[noalloc] refusal o={o} v={v}")
    s, t1, t2, t3p = _state(o, v, seed)
    with binding.Engine(o, v, s["naux"]) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.set_amplitudes(t1, t2, t3p)
        with pytest.raises(binding.CCTError) as e:
            eng.energy_q_noalloc()
        assert e.value.code == binding.CCT_ENOMEM
        assert "MiB" in str(e.value)
        # the context stays usable
        e1 = eng.energy_q()
        assert np.isfinite(e1)
