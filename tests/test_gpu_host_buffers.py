"""Host-memory arguments of the one-shot calls, on an MI355X.

The residual calls accept host arrays (pageable or pinned) as well as device
arrays: host inputs are staged through the workspace and host outputs copied
back.  The kernels are the same, so a call with host arguments must give the
bits of the same call with device arguments; the blocks form is also checked
against the oracle with the (vv|vo)/(vv|ov) blocks passed in several slabs.
"""
import os
import sys

import numpy as np
import pytest

from oracle import cc3_oracle as O
from paper_2007_01088_amd.synth import make_inputs

pytestmark = pytest.mark.gpu
TOL = 1e-11


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx():
    _torch()
    from paper_2007_01088_amd import cc3
    c = cc3.Context(0)
    yield c
    c.close()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def host(torch, d, keys=("eps", "L", "t1", "t2")):
    return {k: torch.from_numpy(np.ascontiguousarray(d[k])) for k in keys}


def same_bits(name, a, b):
    a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
    b = b.cpu().numpy() if hasattr(b, "cpu") else np.asarray(b)
    assert a.shape == b.shape, name
    diff = int(np.count_nonzero(a.view(np.uint64) != b.view(np.uint64)))
    say(f"  {name}: {diff} differing elements of {a.size}")
    assert diff == 0, name


def assert_close(name, got, ref):
    got = np.asarray(got)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    say(f"  {name}: rel2 {err:.3e}")
    assert err <= TOL, (name, err)


@pytest.mark.parametrize("no,nv,nJ", [(4, 20, 60), (5, 37, 50)])
def test_residual_host_equals_device(ctx, no, nv, nJ):
    torch = _torch()
    say(f"host buffers: residual no={no} nv={nv} nchol={nJ}")
    d = make_inputs(no, nv, nJ)
    h = host(torch, d)
    g = {k: v.cuda() for k, v in h.items()}
    d1, d2 = ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"])
    torch.cuda.synchronize()
    h1, h2 = ctx.triples_residual(h["eps"], h["L"], h["t1"], h["t2"])
    assert not h1.is_cuda and not h2.is_cuda
    same_bits("Omega1", h1, d1)
    same_bits("Omega2", h2, d2)
    # pinned host outputs, a mix of host and device inputs
    p1 = torch.empty((no, nv), dtype=torch.float64).pin_memory()
    p2 = torch.empty((no, no, nv, nv), dtype=torch.float64).pin_memory()
    ctx.triples_residual(g["eps"], h["L"], g["t1"], h["t2"], omega1=p1, omega2=p2)
    same_bits("Omega1 pinned", p1, d1)
    same_bits("Omega2 pinned", p2, d2)


def test_accumulate_into_host_outputs(ctx):
    torch = _torch()
    from paper_2007_01088_amd import cc3
    no, nv, nJ = 4, 20, 60
    say(f"host buffers: CC3_ACCUMULATE into host outputs no={no} nv={nv}")
    d = make_inputs(no, nv, nJ)
    h = host(torch, d)
    g = {k: v.cuda() for k, v in h.items()}
    rng = np.random.default_rng(7)
    base1 = rng.standard_normal((no, nv))
    base2 = rng.standard_normal((no, no, nv, nv))
    g1 = torch.from_numpy(base1.copy()).cuda()
    g2 = torch.from_numpy(base2.copy()).cuda()
    ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], omega1=g1, omega2=g2,
                         flags=cc3.ACCUMULATE)
    torch.cuda.synchronize()
    o1 = torch.from_numpy(base1.copy())
    o2 = torch.from_numpy(base2.copy())
    ctx.triples_residual(h["eps"], h["L"], h["t1"], h["t2"], omega1=o1, omega2=o2,
                         flags=cc3.ACCUMULATE)
    same_bits("Omega1", o1, g1)
    same_bits("Omega2", o2, g2)


@pytest.mark.parametrize("slab", [0, 4])
def test_blocks_form_host_slabs(ctx, slab):
    torch = _torch()
    no, nv, nJ = 5, 21, 30
    say(f"host buffers: blocks form no={no} nv={nv}, slabs of {slab or 'all'} first indices")
    d = make_inputs(no, nv, nJ)
    Lt = O.t1_transform(d["L"], d["t1"])
    blk = O.IntegralBlocks(Lt, no, full=True)
    F = O.fock_ov(d["L"], d["t1"])
    args = [blk.full_vvvo(), blk.g_oovo, blk.g_ovov, blk.g_ooov, blk.full_vvov(), F]
    r1, r2 = O.triples_residual_blocks(d["eps"], *args, d["t2"])
    ha = [torch.from_numpy(np.ascontiguousarray(a)) for a in args]
    h = host(torch, d, ("eps", "t2"))
    ga = [a.cuda() for a in ha]
    g1, g2 = ctx.triples_residual_blocks(h["eps"].cuda(), *ga, h["t2"].cuda())
    torch.cuda.synchronize()
    old = os.environ.get("CC3_STAGE_Y")
    if slab:
        os.environ["CC3_STAGE_Y"] = str(slab)  # 21 = 5 slabs of 4 + a ragged slab of 1
    try:
        o1, o2 = ctx.triples_residual_blocks(h["eps"], *ha, h["t2"])
    finally:
        if old is None:
            os.environ.pop("CC3_STAGE_Y", None)
        else:
            os.environ["CC3_STAGE_Y"] = old
    same_bits("Omega1", o1, g1)
    same_bits("Omega2", o2, g2)
    assert_close("Omega1 vs oracle", o1.numpy(), r1)
    assert_close("Omega2 vs oracle", o2.numpy(), r2)


def test_subset_and_t3_block_host(ctx):
    torch = _torch()
    no, nv, nJ = 4, 20, 60
    say(f"host buffers: subset and t3 block no={no} nv={nv}")
    d = make_inputs(no, nv, nJ)
    h = host(torch, d)
    g = {k: v.cuda() for k, v in h.items()}
    tri = [[3, 1, 0], [2, 2, 1], [1, 0, 0]]
    d1, d2 = ctx.triples_residual_subset(g["eps"], g["L"], g["t1"], g["t2"], tri)
    torch.cuda.synchronize()
    o1, o2 = ctx.triples_residual_subset(h["eps"], h["L"], h["t1"], h["t2"], tri)
    assert not o1.is_cuda
    same_bits("Ot1 subset", o1, d1)
    same_bits("Ot2 subset", o2, d2)
    td = ctx.t3_block(g["eps"], g["L"], g["t1"], g["t2"], 2, 0, 1)
    torch.cuda.synchronize()
    th = ctx.t3_block(h["eps"], h["L"], h["t1"], h["t2"], 2, 0, 1)
    assert not th.is_cuda
    same_bits("tau", th, td)


def test_jacobian_prep_rejects_host(ctx):
    torch = _torch()
    from paper_2007_01088_amd import cc3
    no, nv, nJ = 3, 8, 10
    d = make_inputs(no, nv, nJ)
    h = host(torch, d)
    g = {k: v.cuda() for k, v in h.items()}
    zv = torch.empty((nv, nv, no, nv), dtype=torch.float64, device="cuda")
    zo = torch.empty((nv, no, no, no), dtype=torch.float64, device="cuda")
    ws = ctx.workspace(cc3.workspace_size(no, nv, nJ))
    rc = cc3._jprep(ctx._h, no, nv, nJ, h["eps"].data_ptr(), g["L"].data_ptr(),
                    g["t1"].data_ptr(), g["t2"].data_ptr(), zv.data_ptr(), zo.data_ptr(), 0, 0,
                    ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert rc == cc3.E_INVAL
    assert "device memory" in cc3.last_error()
