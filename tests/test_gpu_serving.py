"""The serving loop (cc3_server_*, cc3_submit/cc3_wait) on an MI355X.

Each request's result is checked against the CPU oracle (FP64 bar: 1e-11
relative, per result) and against the same request run alone: the library's
reductions are in a fixed order with no atomics and a request's plan depends
only on its sizes and the server, so a result computed while other requests
share the device is bit-identical to the one computed alone.
"""
import sys

import numpy as np
import pytest

from oracle import cc3_oracle as O
from paper_2007_01088_amd.synth import make_inputs, perturb_t2

pytestmark = pytest.mark.gpu
TOL = 1e-11
MOLS = [(4, 20, 60), (5, 24, 40), (6, 30, 50), (3, 17, 30)]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def data():
    out = []
    for t, (no, nv, nJ) in enumerate(MOLS):
        d = make_inputs(no, nv, nJ, tag=40 + t)
        d["ref"] = O.triples_residual(d["eps"], d["L"], d["t1"], d["t2"])
        out.append(d)
    return out


def make_server(torch, nbytes, slots):
    from paper_2007_01088_amd import cc3
    arena = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    return cc3.Server(arena, max_inflight=slots), cc3


def register_all(torch, srv, data):
    return [srv.register(d["no"], d["nv"], dev(torch, d["eps"]), dev(torch, d["L"]),
                         dev(torch, d["t1"])) for d in data]


def test_mix_equals_alone_and_oracle(data):
    torch = _torch()
    say("serving: 4 molecules, 4 slots, all submitted at once, then each alone")
    srv, cc3 = make_server(torch, 1 << 30, 4)
    mols = register_all(torch, srv, data)
    t2s = [dev(torch, d["t2"]) for d in data]
    tickets = [srv.submit(m, t2) for m, t2 in zip(mols, t2s)]
    mixed = [srv.wait(t, mol=m) for t, m in zip(tickets, mols)]
    st = srv.stats()
    say(f"  stats after the mix: {st}")
    assert st["completed"] == 4 and st["failed"] == 0
    for d, (o1, o2, tm) in zip(data, mixed):
        r1, r2 = d["ref"]
        e1, e2 = rel(o1.cpu().numpy(), r1), rel(o2.cpu().numpy(), r2)
        say(f"  no={d['no']} nv={d['nv']}: rel2 {e1:.2e} {e2:.2e}; timing {tm}")
        assert e1 <= TOL and e2 <= TOL
        assert tm["arrival_s"] <= tm["admit_s"] <= tm["finish_s"]
        assert tm["device_ms"] > 0 and tm["rebuilt"] == 1
    for m, t2, (o1, o2, _) in zip(mols, t2s, mixed):
        a1, a2, tm = srv.wait(srv.submit(m, t2), mol=m)
        assert tm["rebuilt"] == 0  # t1 unchanged: the resident blocks are reused
        assert torch.equal(a1, o1) and torch.equal(a2, o2)
    srv.close()


def test_solver_iterations_closed_loop(data):
    """Closed loop per molecule: perturbed t2 each call, a new t1 on the third call."""
    torch = _torch()
    say("serving: closed-loop iterations with perturbed t2 and one t1 update")
    srv, cc3 = make_server(torch, 1 << 30, 2)
    d = data[1]
    m = srv.register(d["no"], d["nv"], dev(torch, d["eps"]), dev(torch, d["L"]),
                     dev(torch, d["t1"]))
    t2 = d["t2"]
    t1 = d["t1"]
    for it in range(4):
        t2 = perturb_t2(t2, seed=100 + it)
        new_t1 = None
        if it == 2:
            t1 = t1 + 1e-4
            new_t1 = dev(torch, t1)
        o1, o2, tm = srv.wait(srv.submit(m, dev(torch, t2), t1=new_t1), mol=m)
        r1, r2 = O.triples_residual(d["eps"], d["L"], t1, t2)
        e1, e2 = rel(o1.cpu().numpy(), r1), rel(o2.cpu().numpy(), r2)
        say(f"  iteration {it}: rel2 {e1:.2e} {e2:.2e} rebuilt={tm['rebuilt']}")
        assert e1 <= TOL and e2 <= TOL
        assert tm["rebuilt"] == (1 if it in (0, 2) else 0)
    srv.close()


def test_small_arena_admits_one_at_a_time(data):
    """An arena with room for three molecules of one size and a single request's
    workspace: the requests queue and are admitted one by one as memory comes back."""
    torch = _torch()
    d = data[1]
    probe, _ = make_server(torch, 1 << 30, 3)
    res, tr = probe.footprint(d["no"], d["nv"], d["nchol"])
    probe.close()
    nbytes = 3 * res + tr + 256 * 8
    say(f"serving: small arena {nbytes} B (resident {res} x 3, request {tr})")
    srv, _ = make_server(torch, nbytes, 3)
    mols = register_all(torch, srv, [d, d, d])
    tickets = [srv.submit(m, dev(torch, d["t2"])) for m in mols]
    outs = [srv.wait(t, mol=m) for t, m in zip(tickets, mols)]
    st = srv.stats()
    say(f"  stats: {st}")
    assert st["max_inflight_seen"] == 1 and st["completed"] == 3
    assert st["arena_peak"] <= nbytes
    for (o1, o2, tm) in outs:
        assert rel(o1.cpu().numpy(), d["ref"][0]) <= TOL
        assert rel(o2.cpu().numpy(), d["ref"][1]) <= TOL
    # admitted strictly one after the other
    spans = sorted((tm["admit_s"], tm["finish_s"]) for _, _, tm in outs)
    assert all(spans[i][1] <= spans[i + 1][0] for i in range(2))
    srv.close()


def test_mixed_precision_request_matches_oneshot(data):
    torch = _torch()
    from paper_2007_01088_amd import cc3
    d = data[2]
    say("serving: BF16X6 request vs the one-shot call")
    g = {k: dev(torch, d[k]) for k in ("eps", "L", "t1", "t2")}
    ctx = cc3.Context(0)
    ref1, ref2 = ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], prec=cc3.BF16X6)
    torch.cuda.synchronize()
    ctx.close()
    srv, _ = make_server(torch, 1 << 30, 2)
    m = srv.register(d["no"], d["nv"], g["eps"], g["L"], g["t1"])
    o1, o2, _ = srv.wait(srv.submit(m, g["t2"], prec=cc3.BF16X6), mol=m)
    e = rel(o2.cpu().numpy(), ref2.cpu().numpy())
    say(f"  server vs one-shot rel2 {e:.2e}")
    assert e <= 1e-13
    assert rel(o2.cpu().numpy(), d["ref"][1]) <= 1e-7
    srv.close()


def test_host_buffers_and_accumulate(data):
    torch = _torch()
    d = data[0]
    say("serving: host inputs and outputs; CC3_ACCUMULATE into device outputs")
    srv, cc3 = make_server(torch, 1 << 30, 1)
    h = {k: torch.from_numpy(np.ascontiguousarray(d[k])) for k in ("eps", "L", "t1", "t2")}
    m = srv.register(d["no"], d["nv"], h["eps"], h["L"], h["t1"])
    o1 = torch.zeros((d["no"], d["nv"]), dtype=torch.float64)
    o2 = torch.zeros((d["no"],) * 2 + (d["nv"],) * 2, dtype=torch.float64)
    srv.wait(srv.submit(m, h["t2"]), o1, o2)
    assert rel(o1.numpy(), d["ref"][0]) <= TOL and rel(o2.numpy(), d["ref"][1]) <= TOL
    base1 = torch.full((d["no"], d["nv"]), 1e-3, dtype=torch.float64, device="cuda:0")
    base2 = torch.full(tuple(o2.shape), -2e-3, dtype=torch.float64, device="cuda:0")
    srv.wait(srv.submit(m, h["t2"], flags=cc3.ACCUMULATE), base1, base2)
    r1, r2 = d["ref"]
    assert np.linalg.norm(base1.cpu().numpy() - (1e-3 + r1)) <= TOL * np.linalg.norm(r1)
    assert np.linalg.norm(base2.cpu().numpy() - (-2e-3 + r2)) <= TOL * np.linalg.norm(r2)
    with pytest.raises(cc3.CC3Error):  # accumulate needs device outputs
        srv.wait(srv.submit(m, h["t2"], flags=cc3.ACCUMULATE), o1, o2)
    srv.close()


def test_errors_and_cancel(data):
    torch = _torch()
    from paper_2007_01088_amd import cc3
    d = data[0]
    say("serving: error paths")
    srv, _ = make_server(torch, 1 << 30, 1)
    g = {k: dev(torch, d[k]) for k in ("eps", "L", "t1", "t2")}
    m = srv.register(d["no"], d["nv"], g["eps"], g["L"], g["t1"])
    with pytest.raises(cc3.CC3Error) as e:
        srv.submit(m + 999, g["t2"])
    assert e.value.code == cc3.E_NOTFOUND
    with pytest.raises(cc3.CC3Error) as e:
        srv.submit(m, g["t2"], prec=7)
    assert e.value.code == cc3.E_INVAL
    t = srv.submit(m, g["t2"])
    with pytest.raises(cc3.CC3Error) as e:  # one unfinished request per molecule
        srv.submit(m, g["t2"])
    assert e.value.code == cc3.E_BUSY
    with pytest.raises(cc3.CC3Error) as e:
        srv.release(m)
    assert e.value.code == cc3.E_BUSY
    srv.wait(t, mol=m)
    with pytest.raises(cc3.CC3Error) as e:  # collected already
        srv.poll(t)
    assert e.value.code == cc3.E_NOTFOUND
    # a second molecule whose request is queued behind the first one's
    m2 = srv.register(d["no"], d["nv"], g["eps"], g["L"], g["t1"])
    t1_ = srv.submit(m, g["t2"])
    t2_ = srv.submit(m2, g["t2"])
    try:
        srv.cancel(t2_)
        assert srv.wait_status(t2_) == cc3.E_CANCELLED
        say("  cancel: request cancelled while queued")
    except cc3.CC3Error as ex:  # already admitted: it runs to completion
        assert ex.code == cc3.E_BUSY
        assert srv.wait_status(t2_) == cc3.OK
        say("  cancel: request had been admitted already")
    assert srv.wait_status(t1_) == cc3.OK
    # after a cancelled request the blocks are rebuilt on the next one
    o1, o2, tm = srv.wait(srv.submit(m2, g["t2"]), mol=m2)
    assert rel(o2.cpu().numpy(), d["ref"][1]) <= TOL
    srv.release(m2)
    srv.release(m)
    with pytest.raises(cc3.CC3Error) as e:
        srv.release(m)
    assert e.value.code == cc3.E_NOTFOUND
    assert srv.stats()["molecules"] == 0 and srv.stats()["arena_used"] == 0
    srv.close()


def test_request_larger_than_arena(data):
    torch = _torch()
    from paper_2007_01088_amd import cc3
    d = data[2]
    probe, _ = make_server(torch, 1 << 30, 1)
    res, tr = probe.footprint(d["no"], d["nv"], d["nchol"])
    probe.close()
    say(f"serving: arena of {res + 4096} B, request needs {tr}")
    srv, _ = make_server(torch, res + 4096, 1)
    g = {k: dev(torch, d[k]) for k in ("eps", "L", "t1", "t2")}
    m = srv.register(d["no"], d["nv"], g["eps"], g["L"], g["t1"])
    with pytest.raises(cc3.CC3Error) as e:
        srv.submit(m, g["t2"])
    assert e.value.code == cc3.E_NOMEM
    with pytest.raises(cc3.CC3Error) as e:  # no room for a second molecule
        srv.register(d["no"], d["nv"], g["eps"], g["L"], g["t1"])
    assert e.value.code == cc3.E_NOMEM
    srv.close()


# small molecules of the serving mix's size range (no 5-20, nv 60-250), each at most
# 2e12 nominal FLOP, with one to eleven batches
PACK_MOLS = [(5, 60, 195), (8, 100, 324), (10, 90, 300), (6, 150, 468), (12, 120, 396)]


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_packed_group_equals_alone(prec_name):
    """Five small molecules queued behind a large request on one slot run as one packed
    group (batch s of each in the same persistent launches); each result equals, bit for
    bit, the result of the same request run alone with packing off, and the smallest
    one matches the oracle."""
    torch = _torch()
    from paper_2007_01088_amd import cc3
    from paper_2007_01088_amd.synth import make_inputs_device
    prec = {"fp64": cc3.FP64, "fp32": cc3.FP32}[prec_name]
    say(f"packing ({prec_name}): a large request, then {len(PACK_MOLS)} small ones on one slot")
    srv, _ = make_server(torch, 48 << 30, 1)
    srv.set_packing(8, 2e12)
    big = make_inputs_device(12, 160, 516, tag=77)
    mb = srv.register(12, 160, big["eps"], big["L"], big["t1"])
    ds = [make_inputs_device(no, nv, nJ, tag=90 + t) for t, (no, nv, nJ) in enumerate(PACK_MOLS)]
    ms = [srv.register(d["no"], d["nv"], d["eps"], d["L"], d["t1"]) for d in ds]
    torch.cuda.synchronize()
    tb = srv.submit(mb, big["t2"], prec=prec)
    tks = [srv.submit(m, d["t2"], prec=prec) for m, d in zip(ms, ds)]
    srv.wait(tb, want_result=False)
    packed = [srv.wait(t, mol=m) for t, m in zip(tks, ms)]
    st = srv.stats()
    say(f"  stats: packed {st['packed']} in {st['packs']} group(s)")
    assert st["packs"] >= 1 and st["packed"] >= 2, st
    assert len({tm["slot"] for _, _, tm in packed}) == 1
    srv.set_packing(1, 0)
    for (no, nv, _), m, d, (p1, p2, tm) in zip(PACK_MOLS, ms, ds, packed):
        a1, a2, _ = srv.wait(srv.submit(m, d["t2"], prec=prec), mol=m)
        same = torch.equal(a1, p1) and torch.equal(a2, p2)
        say(f"  no={no} nv={nv}: packed == alone bit for bit: {same} "
            f"(device {tm['device_ms']:.1f} ms)")
        assert same
    assert srv.stats()["packs"] == st["packs"]
    # the smallest molecule against the oracle (FP64 bar; FP32-W bound 1e-7)
    d0 = ds[0]
    h = {k: d0[k].cpu().numpy() for k in ("eps", "L", "t1", "t2")}
    r1, r2 = O.triples_residual(h["eps"], h["L"], h["t1"], h["t2"])
    e1, e2 = rel(packed[0][0].cpu().numpy(), r1), rel(packed[0][1].cpu().numpy(), r2)
    say(f"  no=5 nv=60 against the oracle: {e1:.2e} {e2:.2e}")
    bound = TOL if prec_name == "fp64" else 1e-7
    assert e1 <= bound and e2 <= bound
    srv.close()
