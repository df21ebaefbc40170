"""Parity of the transition-density contributions (Algorithm 3) on an MI355X with the
CPU oracle, through the C ABI (cc3_transition_density).

FP64 bar, per result: ||D_gpu - D_oracle||_2 <= 1e-11 ||D_oracle||_2 and the same in
the max norm.  The oracle evaluates the occupied-index loop for D_cd, D_kc, Y^o and
D_ld and, for D_lk, the loop over virtual triples that the paper prints; the device
evaluates D_lk as Gram matrices of the cubes of each occupied pair, so the two D_lk
values come from different loops.  The virtual loop of the oracle is slow (pure
Python over nv^3/6 triples), so the larger sizes compare the occupied-loop results
only.
"""
import sys

import numpy as np
import pytest

from oracle import cc3_oracle as O
from paper_2007_01088_amd.synth import make_inputs, make_left_inputs

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


@pytest.fixture(scope="module")
def ctx():
    torch, cc3 = _setup()
    c = cc3.Context(0)
    yield c
    c.close()


def close(name, got, ref):
    got = np.asarray(got)
    e2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    em = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"  {name}: rel2 {e2:.3e} relmax {em:.3e}")
    assert e2 <= TOL and em <= TOL, (name, e2, em)


def run(ctx, torch, d, lf, flags=0):
    g = {k: torch.from_numpy(np.ascontiguousarray(d[k])).cuda() for k in ("eps", "L", "t1", "t2")}
    l1 = torch.from_numpy(lf["l1"]).cuda()
    l2 = torch.from_numpy(lf["l2"]).cuda()
    out = ctx.transition_density(g["eps"], g["L"], g["t1"], g["t2"], l1, l2, lf["omega"],
                                 flags=flags, want_yo=True)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in out]


def oracle(d, lf, virtual=True):
    no = d["no"]
    Lt = O.t1_transform(d["L"], d["t1"])
    blk = O.IntegralBlocks(Lt, no, full=True)
    F = O.fock_ov(d["L"], d["t1"])
    D_cd, D_kc, D_ld, Y = O.transition_density_occupied(d["eps"], d["t2"], lf["l1"], lf["l2"],
                                                        lf["omega"], blk, F)
    D_lk = (O.transition_density_virtual(d["eps"], d["t2"], lf["l1"], lf["l2"], lf["omega"], blk,
                                         F) if virtual else None)
    return D_cd, D_kc, D_ld, D_lk, Y


@pytest.mark.parametrize("no,nv,nJ,t1z", [(3, 9, 12, False), (4, 20, 30, False),
                                          (4, 20, 30, True), (5, 17, 24, False),
                                          (12, 24, 40, False), (5, 37, 50, False)])
def test_transition_density_parity(ctx, no, nv, nJ, t1z):
    """Every output, D_lk against the oracle's virtual-index loop.  Ragged 8-blocks
    (nv = 9, 17, 37), no = 12 (78 occupied pairs, triples with equal indices in every
    position)."""
    torch, cc3 = _setup()
    say(f"transition density no={no} nv={nv} nchol={nJ} t1_zero={t1z}")
    d = make_inputs(no, nv, nJ, t1_zero=t1z)
    lf = make_left_inputs(no, nv)
    got = run(ctx, torch, d, lf)
    ref = oracle(d, lf)
    for name, a, b in zip(("D_cd", "D_kc", "D_ld", "D_lk", "Y^o"), got, ref):
        close(name, a, b)


def dlk_from_amplitudes(d, lf):
    """D_lk = -1/2 sum over all (i, j, k, l) and a, b, c of L~^{abc}_{ijk} tau^{abc}_{ijl}
    (the sum the virtual-index loop evaluates), written out from the oracle's amplitude
    functions for every ordered occupied triple."""
    no = d["no"]
    Lt = O.t1_transform(d["L"], d["t1"])
    blk = O.IntegralBlocks(Lt, no, full=True)
    F = O.fock_ov(d["L"], d["t1"])
    D = np.zeros((no, no))
    for i in range(no):
        for j in range(no):
            tau = [O.t3_amplitudes(i, j, k, d["eps"], d["t2"], blk) for k in range(no)]
            lt = [O.contravariant(O.l3_amplitudes(i, j, k, lf["omega"], d["eps"], lf["l1"],
                                                  lf["l2"], blk, F)) for k in range(no)]
            for k in range(no):
                for l in range(no):
                    D[l, k] -= 0.5 * float(np.sum(lt[k] * tau[l]))
    return D


@pytest.mark.parametrize("no,nv,nJ", [(4, 130, 40), (16, 16, 24)])
def test_transition_density_larger(ctx, no, nv, nJ):
    """Larger sizes (two 128-wide tiles at nv = 130; 136 occupied pairs at no = 16): the
    occupied-loop outputs against the oracle, and D_lk against its defining sum written
    out from the oracle's t3 and L3 amplitudes of every ordered triple."""
    torch, cc3 = _setup()
    say(f"transition density no={no} nv={nv} nchol={nJ}")
    d = make_inputs(no, nv, nJ)
    lf = make_left_inputs(no, nv)
    got = run(ctx, torch, d, lf)
    ref = oracle(d, lf, virtual=False)
    for name, a, b in zip(("D_cd", "D_kc", "D_ld", "Y^o"), (got[0], got[1], got[2], got[4]),
                          (ref[0], ref[1], ref[2], ref[4])):
        close(name, a, b)
    close("D_lk", got[3], dlk_from_amplitudes(d, lf))


def test_transition_density_edge_cases_and_accumulate(ctx):
    torch, cc3 = _setup()
    # nv = 1: every contravariant amplitude vanishes identically, so does every output
    d = make_inputs(3, 1, 6)
    lf = make_left_inputs(3, 1)
    for x in run(ctx, torch, d, lf):
        assert not np.any(x), x
    # no = 1: only the all-equal triple; no owned triples, and its L~ is zero
    d = make_inputs(1, 7, 6)
    lf = make_left_inputs(1, 7)
    got = run(ctx, torch, d, lf)
    assert not got[0].any() and not got[1].any() and not got[2].any()
    assert np.abs(got[3]).max() < 1e-18
    # CC3_ACCUMULATE adds into the outputs
    no, nv = 3, 9
    d = make_inputs(no, nv, 12)
    lf = make_left_inputs(no, nv)
    base = run(ctx, torch, d, lf)
    g = {k: torch.from_numpy(np.ascontiguousarray(d[k])).cuda() for k in ("eps", "L", "t1", "t2")}
    l1 = torch.from_numpy(lf["l1"]).cuda()
    l2 = torch.from_numpy(lf["l2"]).cuda()
    out = tuple(torch.full(s, 0.25, dtype=torch.float64, device="cuda")
                for s in ((nv, nv), (no, nv), (no, nv), (no, no), (nv, no, no, no)))
    ctx.transition_density(g["eps"], g["L"], g["t1"], g["t2"], l1, l2, lf["omega"],
                           flags=cc3.ACCUMULATE, want_yo=True, out=out)
    torch.cuda.synchronize()
    for a, b in zip(out, base):
        assert np.allclose(a.cpu().numpy() - 0.25, b, rtol=0, atol=1e-15)
    # host memory is refused (by the binding, before the library)
    with pytest.raises(ValueError):
        ctx.transition_density(torch.from_numpy(d["eps"]), g["L"], g["t1"], g["t2"], l1, l2,
                               lf["omega"])
