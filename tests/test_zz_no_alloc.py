"""The allocation-free residual entry point (cc3_triples_residual_noalloc), through the
C ABI, against the workspace entry point cc3_triples_residual on the same inputs.

Both run the same kernels; the allocation-free call may take fewer triples per batch
(to fit the library's static scratch array), which changes only the grouping of the
sums, so the FP64 bar of the parity tests applies: 1e-11 relative per result, in the
2-norm and the max norm.  Two calls in a row, the second with a smaller input, check
that nothing left in the shared array from the first call leaks into the second.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_2007_01088_amd.synth import make_inputs

pytestmark = pytest.mark.gpu
TOL = 1e-11


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_01088_amd import cc3
    return torch, cc3


def _noalloc(cc3, ctx, torch, g, o1, o2, prec=0, flags=0):
    f = cc3._lib.cc3_triples_residual_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int] + \
        [ctypes.c_void_p] * 6 + [ctypes.c_int, ctypes.c_uint, ctypes.c_void_p]
    f.restype = ctypes.c_int
    no, nv = g["t1"].shape
    return f(ctx._h, no, nv, g["L"].shape[0], g["eps"].data_ptr(), g["L"].data_ptr(),
             g["t1"].data_ptr(), g["t2"].data_ptr(), o1.data_ptr(), o2.data_ptr(), prec, flags,
             torch.cuda.current_stream().cuda_stream)


def _close(name, got, ref):
    got, ref = got.cpu().numpy(), ref.cpu().numpy()
    e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    em = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  {name}: rel2 {e2:.3e} relmax {em:.3e}")
    assert e2 <= TOL and em <= TOL, (name, e2, em)


def test_noalloc_matches_workspace_call():
    torch, cc3 = _setup()
    ctx = cc3.Context(0)
    # the second call is smaller than the first; the third needs fewer triples per
    # batch than the workspace call takes, to fit the array
    for no, nv, nJ in ((7, 44, 60), (4, 20, 60), (10, 64, 110)):
        say(f"no-alloc call no={no} nv={nv} nchol={nJ}")
        d = make_inputs(no, nv, nJ)
        g = {k: torch.from_numpy(d[k]).cuda() for k in ("eps", "L", "t1", "t2")}
        r1, r2 = ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"])
        o1 = torch.full((no, nv), float("nan"), dtype=torch.float64, device="cuda")
        o2 = torch.full((no, no, nv, nv), float("nan"), dtype=torch.float64, device="cuda")
        rc = _noalloc(cc3, ctx, torch, g, o1, o2)
        assert rc == 0, cc3.last_error()
        torch.cuda.synchronize()
        _close("Omega1", o1, r1)
        _close("Omega2", o2, r2)
    ctx.close()


def test_noalloc_accumulate_and_errors():
    torch, cc3 = _setup()
    ctx = cc3.Context(0)
    no, nv, nJ = 5, 30, 40
    d = make_inputs(no, nv, nJ)
    g = {k: torch.from_numpy(d[k]).cuda() for k in ("eps", "L", "t1", "t2")}
    r1, r2 = ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"])
    o1 = torch.full((no, nv), 0.5, dtype=torch.float64, device="cuda")
    o2 = torch.full((no, no, nv, nv), -0.25, dtype=torch.float64, device="cuda")
    assert _noalloc(cc3, ctx, torch, g, o1, o2, flags=cc3.ACCUMULATE) == 0, cc3.last_error()
    torch.cuda.synchronize()
    _close("Omega1 + 0.5", o1 - 0.5, r1)
    _close("Omega2 - 0.25", o2 + 0.25, r2)
    # a size whose workspace exceeds the array
    big = make_inputs(12, 120, 400)
    gb = {k: torch.from_numpy(big[k]).cuda() for k in ("eps", "L", "t1", "t2")}
    b1 = torch.empty((12, 120), dtype=torch.float64, device="cuda")
    b2 = torch.empty((12, 12, 120, 120), dtype=torch.float64, device="cuda")
    assert _noalloc(cc3, ctx, torch, gb, b1, b2) == cc3.E_NOMEM
    assert "needs" in cc3.last_error()
    # host memory is refused
    h = {k: torch.from_numpy(d[k]) for k in ("eps", "L", "t1", "t2")}
    assert _noalloc(cc3, ctx, torch, h, o1, o2) == cc3.E_INVAL
    # CC3_CHECK is refused (it would copy to the host and wait)
    assert _noalloc(cc3, ctx, torch, g, o1, o2, flags=cc3.CHECK) == cc3.E_INVAL
    ctx.close()
