"""GPU: device memory through the caller's allocator (cct_alloc_fn / cct_free_fn).

The allocator here is hipMalloc / hipFree of the HIP runtime the library
itself uses, wrapped in Python and counting live blocks.  Results must equal
those of the library's own allocation bit for bit, every block must be
returned at destroy, and a failing allocator must make create return
CCT_ENOMEM with nothing left allocated.
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


def _hip():
    """The libamdhip64 already mapped into this process by libcct."""
    binding.load()
    with open("/proc/self/maps") as f:
        paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert paths, "libamdhip64 is not loaded"
    hip = C.CDLL(sorted(paths)[0])
    hip.hipMalloc.restype = C.c_int
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipFree.restype = C.c_int
    hip.hipFree.argtypes = [C.c_void_p]
    return hip


class CountingAllocator:
    def __init__(self, fail_after=None):
        self.hip = _hip()
        self.live = {}
        self.errors = []
        self.calls = 0
        self.fail_after = fail_after

    def alloc(self, nbytes):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return None
        p = C.c_void_p()
        if self.hip.hipMalloc(C.byref(p), nbytes) != 0:
            return None
        self.live[p.value] = nbytes
        return p.value

    def free(self, ptr):
        # errors are recorded, not raised: an exception cannot leave a C callback
        if ptr not in self.live:
            self.errors.append(f"free of {ptr:#x}, not handed out")
            return
        del self.live[ptr]
        if self.hip.hipFree(C.c_void_p(ptr)) != 0:
            self.errors.append(f"hipFree({ptr:#x}) failed")

    def pair(self):
        return (self.alloc, self.free)


def _system(o, v, seed):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=0.1)
    t1, t2, _ = ci.random_amplitudes(o, v, seed, 0.02, 0.03, 0.0, triples=False)
    return s["f"], s["B"], t1, t2, ci.random_t3_packed(o, v, seed + 100, 0.02)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_engine_with_caller_allocator(prec):
    o, v, seed = 3, 16, 31
    say(f"[allocator] engine prec={prec} o={o} v={v}")
    f, B, t1, t2, t3p = _system(o, v, seed)
    alloc = CountingAllocator()
    results = []
    for allocator in (None, alloc.pair()):
        with binding.Engine(o, v, B.shape[0], precision=prec, allocator=allocator) as eng:
            eng.set_fock(f)
            eng.set_eri_df(B)
            eng.set_amplitudes(t1, t2, t3p)
            r = eng.residual()
            e, _ = eng.update()
            results.append((r, e))
            if allocator is not None:
                say(f"  {len(alloc.live)} blocks, {sum(alloc.live.values()) / 1e6:.1f} MB live")
                assert alloc.live and sum(alloc.live.values()) > 0
    assert not alloc.live, "blocks left after destroy"
    assert not alloc.errors, alloc.errors
    (ra, ea), (rb, eb) = results
    for x, y in zip(ra[:3], rb[:3]):
        assert np.array_equal(x, y)
    assert ea == eb


def test_batch_and_slab_with_caller_allocator():
    say("[allocator] batch and slab")
    sizes = [(3, 12, 30), (4, 10, 28)]
    systems = [ci.make_system(o, v, na, 500 + k, sigma=0.1) for k, (o, v, na) in enumerate(sizes)]
    alloc = CountingAllocator()
    hip = alloc.hip
    hip.hipStreamCreate.restype = C.c_int
    hip.hipStreamCreate.argtypes = [C.POINTER(C.c_void_p)]
    hip.hipStreamDestroy.restype = C.c_int
    hip.hipStreamDestroy.argtypes = [C.c_void_p]
    stream = C.c_void_p()
    assert hip.hipStreamCreate(C.byref(stream)) == 0
    energies = []
    for allocator, st in ((None, None), (alloc.pair(), stream.value)):
        with binding.Batch(sizes, opts={"streams": 2}, stream=st, allocator=allocator) as b:
            for k, s in enumerate(systems):
                b.set_system(k, s["f"], s["B"])
            e, _ = b.iterate(2)
            energies.append(e)
    assert not alloc.live and not alloc.errors
    # the caller's stream outlives the batch (the library does not destroy it)
    assert hip.hipStreamDestroy(stream) == 0
    assert np.array_equal(energies[0], energies[1])

    o, v, naux, first, count = 3, 12, 30, 2, 5
    s = systems[0]
    _, t2, _ = ci.random_amplitudes(o, v, 7, 0.0, 0.03, 0.0, triples=False)
    rng = np.random.default_rng(8)
    Fvv = rng.normal(0, 0.1, (v, v))
    Wt = rng.normal(0, 0.01, (o, v, v, v))
    Wvooo = rng.normal(0, 0.01, (v, o, o, o))
    t3 = ci.random_t3_packed(o, v, 9, 0.02)[first:first + count]
    out = []
    for allocator in (None, alloc.pair()):
        with binding.Slab(o, v, naux, first, count, allocator=allocator) as sl:
            sl.set_intermediates(s["B"], t2, Fvv, Wt, Wvooo)
            sl.set_t3(t3)
            r, n2 = sl.residual()
            out.append(r)
    assert not alloc.live and not alloc.errors
    assert np.array_equal(out[0], out[1])


def test_failing_allocator_gives_enomem_and_leaks_nothing():
    say("[allocator] failing allocator")
    for fail_after in (0, 5):
        alloc = CountingAllocator(fail_after=fail_after)
        with pytest.raises(binding.CCTError) as ei:
            binding.Engine(3, 12, 30, allocator=alloc.pair())
        assert ei.value.code == binding.CCT_ENOMEM
        assert not alloc.live and not alloc.errors


def test_energy_q_scratch_through_caller_allocator():
    """cct_energy_q takes its scratch (bare integrals, Wbar, unpacked T3, the
    task blocks) from the caller's allocator and returns every block before it
    returns; the energy equals the library-allocated one bit for bit."""
    o, v, seed = 3, 10, 41
    say(f"[allocator] energy_q o={o} v={v}")
    f, B, t1, t2, t3p = _system(o, v, seed)
    alloc = CountingAllocator()
    out = []
    for allocator in (None, alloc.pair()):
        with binding.Engine(o, v, B.shape[0], allocator=allocator) as eng:
            eng.set_fock(f)
            eng.set_eri_df(B)
            eng.set_amplitudes(t1, t2, t3p)
            before = dict(alloc.live)
            calls = alloc.calls
            out.append(eng.energy_q(tasks=True))
            if allocator is not None:
                assert alloc.calls > calls, "no scratch came from the caller's allocator"
                assert alloc.live == before, "energy_q left scratch blocks allocated"
    assert not alloc.live and not alloc.errors
    (ea, ta), (eb, tb) = out
    assert ea == eb and np.array_equal(ta, tb)
