"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/cct.h, and its host-only entry points behave."""

import os
import re
import subprocess

import pytest

from paper_2607_00981_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "cct.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cct_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _declared()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cct_\w+)", out))
    for name in names:
        assert name in exported, name
        assert hasattr(lib, name)


def test_packed_index_matches_enumeration():
    for o in (1, 2, 5, 9):
        idx = 0
        for i in range(o):
            for j in range(i, o):
                for k in range(j, o):
                    assert binding.packed_index(o, i, j, k) == idx
                    idx += 1
        assert idx == binding.ntri(o)
    assert binding.packed_index(4, 2, 1, 3) == -1
    assert binding.packed_index(4, 0, 0, 4) == -1
    assert binding.packed_index(0, 0, 0, 0) == -1


def test_strerror_codes():
    lib = binding.load()
    assert lib.cct_strerror(0) == b"ok"
    assert lib.cct_strerror(-2) == b"out of device memory"
    assert lib.cct_strerror(-6) == b"not converged"
    assert lib.cct_strerror(5) == b"unknown error"


def test_create_rejects_bad_arguments():
    import ctypes as C
    lib = binding.load()
    h = C.c_void_p()
    assert lib.cct_create(0, 10, 10, 0, None, None, None, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 7, None, None, None, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 0, b'{"diis_t3": "bogus"}', None, None, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 0, None, None, None, None, None, None) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 0, b'{"tol": -1}', None, None, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 0, b'{"diis_t3": "subspace:11"}', None, None, None, None,
                          C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 0, b'{"diis_t3": "subspace:0"}', None, None, None, None,
                          C.byref(h)) == binding.CCT_EINVAL
    lib.cct_destroy(None)


def test_create_rejects_half_an_allocator():
    """The caller's allocator comes as a pair: alloc without free (or free
    without alloc) is refused before any device call, for every create."""
    import ctypes as C
    lib = binding.load()
    h = C.c_void_p()
    a_cb = binding.ALLOC_FN(lambda n, u: None)
    f_cb = binding.FREE_FN(lambda p, u: None)
    a, f = C.cast(a_cb, C.c_void_p), C.cast(f_cb, C.c_void_p)
    assert lib.cct_create(2, 10, 10, 0, None, a, None, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_create(2, 10, 10, 0, None, None, f, None, None, C.byref(h)) == binding.CCT_EINVAL
    sizes = (C.c_int * 1)(2)
    assert lib.cct_batch_create(1, sizes, sizes, sizes, 0, None, a, None, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert lib.cct_slab_create(2, 10, 10, 0, 1, 0, None, None, f, None, None, C.byref(h)) == binding.CCT_EINVAL
    assert not h.value


def test_q_task_count_formula():
    for o in range(0, 12):
        n = sum(1 for i in range(o) for j in range(i, o) for k in range(j, o) for l in range(k, o))
        assert binding.q_task_count(o) == n
    assert binding.q_task_count(-1) == -1


def test_q_task_count_reproduces_the_papers_printed_counts():
    import math
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(ROOT, "tests", "golden", "q_task_counts.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for v, blk, n, tasks in rows:
        assert math.ceil(v / blk) == n
        assert binding.q_task_count(n) == tasks


def test_quad_packed_index_matches_enumeration():
    """cct_quad_packed_index / cct_quad_count (host only) against the
    lexicographic enumeration of i <= j <= k <= l."""
    from oracle import rccsdtq as Q4

    lib = binding.load()
    for o in (1, 2, 3, 5):
        lst = Q4.packed_list4(o)
        assert binding.quad_count(o) == len(lst) == o * (o + 1) * (o + 2) * (o + 3) // 24
        for n, q in enumerate(lst):
            assert lib.cct_quad_packed_index(o, *q) == n
    assert lib.cct_quad_packed_index(3, 0, 1, 0, 2) == -1
    assert lib.cct_quad_packed_index(3, 0, 0, 1, 3) == -1
    assert binding.quad_count(-1) == -1


def test_q_abc_task_count_is_the_tile_quadruple_count():
    import itertools
    for v, nb in ((1, 1), (7, 2), (8, 4), (180, 4), (90, 8), (30, 16)):
        nt = -(-v // nb)
        assert binding.q_abc_task_count(v, nb) == sum(1 for _ in itertools.combinations_with_replacement(range(nt), 4))
    assert binding.q_abc_task_count(0, 4) == -1
    assert binding.q_abc_task_count(10, 0) == -1
