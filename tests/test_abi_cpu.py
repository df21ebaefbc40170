"""CPU-side checks of the C ABI library: it loads, exports every symbol the
header declares, and its host-only entry points validate their arguments.
No compute call is made here (no GPU in this environment)."""
import ctypes
import os
import re
from math import comb

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2007_01088_amd", "libcc3.so")
HEADER = os.path.join(ROOT, "include", "cc3.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(cc3_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libcc3.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert "cc3_triples_residual" in syms and len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_names_match_header():
    from paper_2007_01088_amd import cc3
    assert set(cc3.EXPORTED) <= set(declared_symbols())


def test_workspace_size_and_validation(lib):
    f = lib.cc3_workspace_size
    f.argtypes = [ctypes.c_int] * 4 + [ctypes.c_uint, ctypes.POINTER(ctypes.c_size_t)]
    n = ctypes.c_size_t(0)
    assert f(12, 120, 400, 0, 0, ctypes.byref(n)) == 0
    nv, no = 120, 12
    # at least the resident blocks: two nv^3 no slabs and the contravariant doubles residual
    assert n.value >= (2 * no * nv**3 + no * no * nv * nv) * 8
    assert f(0, 120, 400, 0, 0, ctypes.byref(n)) == -1
    assert f(12, -1, 400, 0, 0, ctypes.byref(n)) == -1
    assert f(12, 120, -5, 0, 0, ctypes.byref(n)) == -1
    assert f(12, 120, 400, 99, 0, ctypes.byref(n)) == -1
    assert f(12, 120, 400, 0, 0, None) == -1
    lib.cc3_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.cc3_last_error()


def test_flops_counts(lib):
    f = lib.cc3_flops
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                  ctypes.POINTER(ctypes.c_double)]
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    for no, nv in [(4, 20), (12, 120), (31, 400)]:
        assert f(no, nv, ctypes.byref(a), ctypes.byref(b)) == 0
        assert a.value == 4.0 * nv**4 * no**3
        # the library builds 6 W terms per distinct triple and 3 when two indices are
        # equal (the other three repeat), and contracts each distinct permutation once
        D, E = comb(no, 3), no * (no - 1)
        w = 2 * nv**4 + 2 * nv**3 * no
        perm = 2 * nv**4 + 2 * nv**3 + 2 * nv**3 + 2 * nv**3 * no
        assert b.value == pytest.approx((6 * D + 3 * E) * (w + perm), rel=1e-14)
        # its dominant part is 4 nv^4 (no^3 - no)
        assert (6 * D + 3 * E) * 4 * nv**4 == 4 * nv**4 * (no**3 - no)
    assert f(0, 3, ctypes.byref(a), ctypes.byref(b)) == -1


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib.cc3_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    h = ctypes.c_void_p()
    rc = lib.cc3_create(ctypes.byref(h), 0)
    assert rc in (-1, -3)


def test_product_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2007_01088_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text, fn
                assert "cc3_oracle" not in text and "bruteforce" not in text, fn


def test_serving_calls_validate_without_a_device(lib):
    """Null server handles and null out-pointers are rejected before any HIP call."""
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.cc3_server_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.c_int]
    assert lib.cc3_server_create(None, 0, None, 0, 1) == -1
    h = ctypes.c_void_p()
    assert lib.cc3_server_create(ctypes.byref(h), 0, None, 1 << 20, 0) == -1  # max_inflight
    assert lib.cc3_server_create(ctypes.byref(h), 0, None, 1 << 20, 9) == -1
    lib.cc3_server_footprint.argtypes = [ctypes.c_void_p] + [ctypes.c_int] * 4 + [
        ctypes.c_void_p, ctypes.c_void_p]
    assert lib.cc3_server_footprint(None, 4, 20, 60, 0, None, None) == -1
    lib.cc3_submit.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, u64p]
    assert lib.cc3_submit(None, 1, None, None, 0, 0, None) == -1
    lib.cc3_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    assert lib.cc3_poll(None, 1, None) == -1
    lib.cc3_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64] + [ctypes.c_void_p] * 3
    assert lib.cc3_wait(None, 1, None, None, None) == -1
    lib.cc3_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    assert lib.cc3_cancel(None, 1) == -1
    lib.cc3_molecule_release.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    assert lib.cc3_molecule_release(None, 1) == -1
    lib.cc3_server_get_stats.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.cc3_server_get_stats(None, None) == -1
    lib.cc3_server_destroy.argtypes = [ctypes.c_void_p]
    assert lib.cc3_server_destroy(None) == 0
