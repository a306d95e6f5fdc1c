"""Error behaviour of the C ABI on a GPU: invalid arguments, calls in the
wrong state and unsupported term masks return the documented codes and leave
the context usable."""

import numpy as np
import pytest

import cct_inputs as ci
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu


def test_state_and_argument_errors_single():
    o, v, naux = 2, 6, 16
    with binding.Engine(o, v, naux) as eng:
        with pytest.raises(binding.CCTError) as e:
            eng.residual()
        assert e.value.code == binding.CCT_ESTATE
        s = ci.make_system(o, v, naux, 3)
        eng.set_fock(s["f"])
        with pytest.raises(binding.CCTError) as e:
            eng.update()
        assert e.value.code == binding.CCT_ESTATE
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        e1, _ = eng.update()
        assert np.isfinite(e1)
        lib = binding.load()
        assert lib.cct_copy_r3(eng.h, -1, 1, binding._ptr(np.empty(1))) == binding.CCT_EINVAL
        assert lib.cct_autotune(eng.h, -1.0, None) == binding.CCT_EINVAL
        assert lib.cct_solve(eng.h, 0, 1e-8, None, None) == binding.CCT_EINVAL
    lib = binding.load()
    h = binding.C.c_void_p()
    assert lib.cct_create(0, 5, 10, 0, None, None, None, None, None, binding.C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 5, 10, 7, None, None, None, None, None, binding.C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 5, 10, 0, b'{"diis_t3": "sometimes"}', None, None, None, None, binding.C.byref(h)) == binding.CCT_EINVAL


def test_slab_and_batch_errors():
    lib = binding.load()
    h = binding.C.c_void_p()
    # slab range beyond the packed triples of o = 3 (10 triples)
    assert lib.cct_slab_create(3, 8, 20, 8, 4, 0, None, None, None, None, None, binding.C.byref(h)) == binding.CCT_EINVAL
    with binding.Slab(3, 8, 20, 0, 4) as sl:
        with pytest.raises(binding.CCTError) as e:
            sl.residual()
        assert e.value.code == binding.CCT_ESTATE
        with pytest.raises(binding.CCTError) as e:
            sl.residual(("RA",))
        assert e.value.code == binding.CCT_EINVAL
    with pytest.raises(binding.CCTError):
        binding.Batch([(2, 6, 16)], opts={"streams": 17})
    with binding.Batch([(2, 6, 16), (3, 7, 20)]) as b:
        with pytest.raises(binding.CCTError) as e:
            b.iterate(1)
        assert e.value.code == binding.CCT_ESTATE
