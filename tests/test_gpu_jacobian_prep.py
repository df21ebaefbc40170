"""Parity of the Jacobian-preparation intermediates (Algorithm 2) on an MI355X with
the CPU oracle, through the C ABI (cc3_jacobian_prep).

FP64 bar: 1e-11 relative per result (2-norm and max), as for the residual.  At the
benchmark size, where the oracle would take minutes, the intermediates are checked
by properties: sum_j Z~o_{ajij} equals the contravariant Omega1 of the residual
path, and the intermediates are linear in t2.
"""
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


def dev(torch, d):
    return {k: torch.from_numpy(np.ascontiguousarray(d[k])).cuda() for k in ("eps", "L", "t1", "t2")}


def close(name, got, ref, tol=TOL):
    got = np.asarray(got)
    e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    em = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  {name}: rel2 {e2:.3e} relmax {em:.3e}")
    assert e2 <= tol and em <= tol, (name, e2, em)


@pytest.mark.parametrize("no,nv,nJ,t1z", [(4, 20, 60, False), (4, 20, 60, True), (3, 9, 12, False),
                                          (5, 37, 50, False), (6, 130, 40, False),
                                          (16, 16, 40, False), (20, 12, 30, False),
                                          (35, 8, 16, False), (3, 196, 24, False)])
def test_jacobian_prep_parity(ctx, no, nv, nJ, t1z):
    """(16, 16): batches of 160 triples in which one occupied index heads up to 255
    (triple, permutation) pairs, beyond half the per-index list bound.  (20, 12) and
    (35, 8): the Zo partials span two and three 16-wide tiles of l.  (3, 196): above
    nv = 192, where the batches run on one stream."""
    torch = _torch()
    say(f"jacobian prep no={no} nv={nv} nJ={nJ} t1_zero={t1z}")
    d = make_inputs(no, nv, nJ, t1_zero=t1z)
    rv, ro = O.jacobian_prep(d["eps"], d["L"], d["t1"], d["t2"])
    g = dev(torch, d)
    zv, zo = ctx.jacobian_prep(g["eps"], g["L"], g["t1"], g["t2"])
    torch.cuda.synchronize()
    close("Zv", zv.cpu().numpy(), rv)
    close("Zo", zo.cpu().numpy(), ro)


def test_jacobian_prep_accumulate_and_mixed(ctx):
    torch = _torch()
    from paper_2007_01088_amd import cc3
    no, nv, nJ = 5, 24, 40
    d = make_inputs(no, nv, nJ)
    rv, ro = O.jacobian_prep(d["eps"], d["L"], d["t1"], d["t2"])
    g = dev(torch, d)
    zv = torch.full((nv, nv, no, nv), 1e-3, dtype=torch.float64, device="cuda")
    zo = torch.full((nv, no, no, no), -2e-3, dtype=torch.float64, device="cuda")
    ctx.jacobian_prep(g["eps"], g["L"], g["t1"], g["t2"], zv, zo, flags=cc3.ACCUMULATE)
    torch.cuda.synchronize()
    close("Zv accumulate", zv.cpu().numpy() - 1e-3, rv, 1e-10)
    close("Zo accumulate", zo.cpu().numpy() + 2e-3, ro, 1e-10)
    for name, prec, bound in (("fp32", cc3.FP32, 1e-7), ("bf16x6", cc3.BF16X6, 1e-7),
                              ("bf16x3", cc3.BF16X3, 3e-5)):
        zv, zo = ctx.jacobian_prep(g["eps"], g["L"], g["t1"], g["t2"], prec=prec)
        torch.cuda.synchronize()
        ev = np.linalg.norm(zv.cpu().numpy() - rv) / np.linalg.norm(rv)
        eo = np.linalg.norm(zo.cpu().numpy() - ro) / np.linalg.norm(ro)
        say(f"  {name}: rel err Zv {ev:.3e} Zo {eo:.3e}")
        assert ev <= bound and eo <= bound


def test_jacobian_prep_properties_at_benchmark_size(ctx):
    torch = _torch()
    no, nv, nJ = 12, 120, 400
    say(f"jacobian prep properties no={no} nv={nv}")
    d = make_inputs(no, nv, nJ)
    g = dev(torch, d)
    zv, zo = ctx.jacobian_prep(g["eps"], g["L"], g["t1"], g["t2"])
    allt = np.array(O.unordered_triples(no), dtype=np.int32)
    o1, _ = ctx.triples_residual_subset(g["eps"], g["L"], g["t1"], g["t2"], allt)
    torch.cuda.synchronize()
    tr = torch.einsum("ajij->ia", zo)
    close("sum_j Zo_ajij vs Omega1~", tr.cpu().numpy(), o1.cpu().numpy())
    zv2, zo2 = ctx.jacobian_prep(g["eps"], g["L"], g["t1"], (2.0 * g["t2"]).contiguous())
    torch.cuda.synchronize()
    close("Zv(2 t2) / 2", (zv2 / 2).cpu().numpy(), zv.cpu().numpy())
    close("Zo(2 t2) / 2", (zo2 / 2).cpu().numpy(), zo.cpu().numpy())
