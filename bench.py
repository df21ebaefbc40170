"""Benchmark of the CC3 ground-state triples residual on one MI355X.

A step is one whole residual evaluation (T1 transformation of the Cholesky
vectors, integral-block build, the restricted triple loop, the covariant
back-transformation) on seeded synthetic inputs already resident in HBM.
The metric is the paper's nominal 4 nv^4 no^3 FLOP per call divided by the
measured time per call.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mixed]

The default workload is no=23 nv=250 nchol=800, the largest size whose timed
calls fit a run of a few minutes (one FP64 call takes about 5 s); the extra
measurements after the timed region (standalone kernel durations, the mixed
precisions, the Jacobian preparation, the CVS worklist, host buffers) take
--extra-steps calls each.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (no, nv, nchol)
    "small": (4, 20, 60),
    "medium": (12, 120, 400),
    "mixed": (23, 250, 800),
    "large": (31, 400, 1200),
}
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6}
DOMINANT_SOURCES = {"w_build": "kern_triples.hip", "omega_contract": "kern_triples.hip",
                    "mix": "kern_triples.hip"}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def source_sha(fn: str) -> str:
    p = os.path.join(ROOT, "paper_2007_01088_amd", "csrc", fn)
    h = hashlib.sha256()
    for part in (p, os.path.join(ROOT, "paper_2007_01088_amd", "csrc", "cc3_device.hpp")):
        with open(part, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha") != source_sha(DOMINANT_SOURCES.get(kernel, "kern_triples.hip")):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(no: int, nv: int, nchol: int, budget_s: float) -> dict:
    """The oracle, as it stands, on a bounded seeded sample of the same workload's triples,
    extrapolated to one whole call by the exact per-triple cost weights."""
    from oracle import cc3_oracle as O
    from paper_2007_01088_amd.synth import make_inputs, sample_triples
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(x.get("num_threads", 1)) for x in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    d = make_inputs(no, nv, nchol)
    t0 = time.perf_counter()
    Lt = O.t1_transform(d["L"], d["t1"])
    blk = O.IntegralBlocks(Lt, no, full=True)
    F = O.fock_ov(d["L"], d["t1"])
    t_prep = time.perf_counter() - t0
    alltri = O.unordered_triples(no)

    def weight(t):  # oracle cost: six W terms, six or three permutations
        i, j, k = t
        return 6 + (6 if len({i, j, k}) == 3 else 3)

    order = sample_triples(no, len(alltri), seed=17)
    done_w, t_loop, n = 0.0, 0.0, 0
    for t in order:
        t = tuple(int(x) for x in t)
        s = time.perf_counter()
        O.omega_tilde(d["eps"], d["t2"], blk, F, triples=[t])
        t_loop += time.perf_counter() - s
        done_w += weight(t)
        n += 1
        if t_loop + t_prep >= budget_s:
            break
    total_w = sum(weight(t) for t in alltri)
    t_call = t_prep + t_loop * total_w / done_w
    nominal = O.nominal_flops(no, nv)
    cpu = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": nominal / t_call / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "cpu": cpu, "host_cpus": os.cpu_count(),
            "sample": f"{n} of {len(alltri)} unordered triples (seeded) plus the full integral "
                      f"preparation, {t_prep + t_loop:.1f} s measured, extrapolated to one call "
                      f"({t_call:.1f} s) by per-triple cost weights",
            "seconds_per_call": t_call}


PREC_NAMES = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}


def _pct(x, q):
    return float(np.percentile(np.asarray(x), q)) if len(x) else None


def serve(n_mol: int, n_calls: int, prec_name: str, slots: int, load: float,
          small_arena_gb: float, seed: int = 5, max_pack: int = 8,
          pack_flops: float = 2e12) -> dict:
    """Serving mix: molecules with no ~ U[5,20], nv ~ U[60,250], Cholesky rank
    3(no+nv), each issuing `n_calls` closed-loop residual calls (the next call
    goes out when the previous result is back, with t2 perturbed as by a solver
    iteration); first calls arrive as a Poisson process at `load` times the
    capacity measured in a saturating run.  Everything goes through the
    library's serving loop (arena admission, concurrent slots)."""
    import torch

    from paper_2007_01088_amd import cc3
    from paper_2007_01088_amd.synth import (make_inputs_device, perturb_t2_device,
                                            poisson_arrivals, serving_mix)
    prec = PREC_NAMES[prec_name]
    mix = serving_mix(n_mol, seed)
    nominal = [cc3.flops(no, nv)[0] for no, nv, _ in mix]
    dev = "cuda:0"
    free, _ = torch.cuda.mem_get_info()
    t2_bytes = sum(no * no * nv * nv * 8 for no, nv, _ in mix)
    arena_bytes = int((free - 2 * t2_bytes - (24 << 30)) * 0.9) & ~255
    log(f"serving: {n_mol} molecules x {n_calls} calls, prec {prec_name}, {slots} slots, "
        f"arena {arena_bytes / 2**30:.1f} GiB")
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
    srv = cc3.Server(arena, max_inflight=slots)
    srv.set_packing(max_pack, pack_flops)
    mols, t2s = [], []
    resident = 0
    for m, (no, nv, nJ) in enumerate(mix):
        d = make_inputs_device(no, nv, nJ, tag=1000 + m, device=dev)
        mols.append(srv.register(no, nv, d["eps"], d["L"], d["t1"]))
        t2s.append(d["t2"])
        resident += srv.footprint(no, nv, nJ, prec)[0]
        del d
    torch.cuda.synchronize()
    log(f"serving: registered {n_mol} molecules, {resident / 2**30:.1f} GiB resident")
    # warm-up call: loads the code objects and creates the slot streams
    srv.wait(srv.submit(mols[0], t2s[0], prec=prec), want_result=False)

    def finish_all(tickets):
        out = {}
        for t, m in tickets.items():
            _, _, tm = srv.wait(t, want_result=False)
            out[m] = tm
        return out

    # capacity: every molecule submits one call at once
    tks = {srv.submit(mols[m], t2s[m], prec=prec): m for m in range(n_mol)}
    tms = finish_all(tks)
    t_first = min(tm["arrival_s"] for tm in tms.values())
    t_last = max(tm["finish_s"] for tm in tms.values())
    cap_rps = n_mol / (t_last - t_first)
    cap_tflops = sum(nominal) / (t_last - t_first) / 1e12
    log(f"serving: saturated capacity {cap_rps:.2f} requests/s, {cap_tflops:.2f} TFLOP/s")

    # Poisson arrivals of first calls at `load` x capacity, then closed loops
    lam = load * cap_rps / n_calls
    arr = poisson_arrivals(n_mol, lam, seed)
    calls_left = [n_calls] * n_mol
    pending = {}
    lat, lat_host, qwait, dev_ms, fin, arr_s, flop_done = [], [], [], [], [], [], 0.0
    t0 = time.perf_counter()
    nxt = 0
    done = 0
    last_log = t0
    it_seed = 0
    while done < n_mol * n_calls:
        now = time.perf_counter() - t0
        while nxt < n_mol and arr[nxt] <= now:
            t = srv.submit(mols[nxt], t2s[nxt], prec=prec)
            pending[t] = (nxt, time.perf_counter())
            nxt += 1
        for t in [t for t in pending if srv.poll(t)]:
            m, t_issue = pending.pop(t)
            _, _, tm = srv.wait(t, want_result=False)
            lat_host.append(time.perf_counter() - t_issue)
            lat.append(tm["finish_s"] - tm["arrival_s"])
            qwait.append(tm["admit_s"] - tm["arrival_s"])
            dev_ms.append(tm["device_ms"])
            fin.append(tm["finish_s"])
            arr_s.append(tm["arrival_s"])
            flop_done += nominal[m]
            done += 1
            calls_left[m] -= 1
            if calls_left[m] > 0:
                it_seed += 1
                t2s[m] = perturb_t2_device(t2s[m], seed=it_seed)
                t = srv.submit(mols[m], t2s[m], prec=prec)
                pending[t] = (m, time.perf_counter())
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            log(f"serving: {done}/{n_mol * n_calls} calls done")
        time.sleep(0.0002)
    makespan = max(fin) - min(arr_s)
    st = srv.stats()
    res = {
        "molecules": n_mol, "calls_per_molecule": n_calls, "requests": n_mol * n_calls,
        "reading": "closed loop per molecule (next call when the previous result is back, "
                   "t2 perturbed by N(0,1e-4^2)), Poisson first arrivals",
        "prec": prec_name, "slots": slots, "arena_gib": arena_bytes / 2**30,
        "resident_gib": resident / 2**30,
        "capacity_requests_per_s": cap_rps, "capacity_tflops": cap_tflops,
        "arrival_rate_molecules_per_s": lam, "load": load,
        "p50_ms": _pct(lat, 50) * 1e3, "p99_ms": _pct(lat, 99) * 1e3,
        "p50_ms_host": _pct(lat_host, 50) * 1e3, "p99_ms_host": _pct(lat_host, 99) * 1e3,
        "queue_wait_p50_ms": _pct(qwait, 50) * 1e3, "queue_wait_p99_ms": _pct(qwait, 99) * 1e3,
        "device_ms_p50": _pct(dev_ms, 50), "device_ms_p99": _pct(dev_ms, 99),
        "aggregate_tflops": flop_done / makespan / 1e12, "makespan_s": makespan,
        "max_inflight_seen": st["max_inflight_seen"], "arena_peak_gib": st["arena_peak"] / 2**30,
        "packing": {"max_pack": max_pack, "max_request_flops": pack_flops,
                    "requests_packed": st["packed"], "groups": st["packs"]},
    }
    log(f"serving: p50 {res['p50_ms']:.1f} ms p99 {res['p99_ms']:.1f} ms, "
        f"{res['aggregate_tflops']:.2f} TFLOP/s aggregate")
    srv.close()
    del arena
    torch.cuda.empty_cache()

    if small_arena_gb > 0:
        # admission under memory pressure: a small arena, molecules that fit, all at once
        nbytes = int(small_arena_gb * 2**30) & ~255
        arena = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        srv = cc3.Server(arena, max_inflight=slots)
        srv.set_packing(max_pack, pack_flops)
        sub, used, tr_max = [], 0, 0
        for m, (no, nv, nJ) in enumerate(mix):
            r, tr = srv.footprint(no, nv, nJ, prec)
            if used + r + max(tr_max, tr) <= nbytes * 0.98:
                sub.append(m)
                used += r
                tr_max = max(tr_max, tr)
        ids = {}
        for m in sub:
            no, nv, nJ = mix[m]
            d = make_inputs_device(no, nv, nJ, tag=1000 + m, device=dev)
            ids[m] = srv.register(no, nv, d["eps"], d["L"], d["t1"])
            del d
        tks = {srv.submit(ids[m], t2s[m], prec=prec): m for m in sub}
        tms = finish_all(tks)
        st = srv.stats()
        lat_s = [tm["finish_s"] - tm["arrival_s"] for tm in tms.values()]
        q_s = [tm["admit_s"] - tm["arrival_s"] for tm in tms.values()]
        span = max(tm["finish_s"] for tm in tms.values()) - min(tm["arrival_s"] for tm in tms.values())
        res["small_arena"] = {
            "arena_gib": nbytes / 2**30, "molecules": len(sub), "resident_gib": used / 2**30,
            "largest_request_gib": tr_max / 2**30, "submitted_at_once": len(sub),
            "max_inflight_seen": st["max_inflight_seen"], "arena_peak_gib": st["arena_peak"] / 2**30,
            "p50_ms": _pct(lat_s, 50) * 1e3, "p99_ms": _pct(lat_s, 99) * 1e3,
            "queue_wait_p50_ms": _pct(q_s, 50) * 1e3, "queue_wait_p99_ms": _pct(q_s, 99) * 1e3,
            "aggregate_tflops": sum(nominal[m] for m in sub) / span / 1e12,
        }
        log(f"serving, small arena: {len(sub)} molecules, max in flight "
            f"{st['max_inflight_seen']}, p99 {res['small_arena']['p99_ms']:.1f} ms")
        srv.close()
        del arena
        torch.cuda.empty_cache()
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed", choices=sorted(WORKLOADS))
    ap.add_argument("--extra-steps", type=int, default=2,
                    help="timed calls of each extra measurement after the timed region")
    ap.add_argument("--prec", default="fp64", choices=["fp64"])
    ap.add_argument("--mixed-forms", default="fp32,bf16x6,bf16x3,fp32_all,bf16x6_all,bf16x3_all",
                    help="comma-separated low-precision forms to time after the FP64 steps")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip timing the mixed-precision W contractions (FP32, BF16x3, BF16x6)")
    ap.add_argument("--no-jacobian-prep", action="store_true",
                    help="skip timing the Jacobian-preparation intermediates (Algorithm 2)")
    ap.add_argument("--standalone-steps", type=int, default=2,
                    help="calls with CC3_ONE_STREAM after the timed region, for kernel durations "
                         "without batch overlap (0: skip)")
    ap.add_argument("--no-cvs", action="store_true", help="skip the CVS worklist timing")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the Algorithm 3 (transition-density) timing")
    ap.add_argument("--no-host-buffers", action="store_true",
                    help="skip the timing of the call with host-memory arrays")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-molecules", type=int, default=16,
                    help="serving mix size (0 skips the serving measurement)")
    ap.add_argument("--serve-calls", type=int, default=2, help="closed-loop calls per molecule")
    ap.add_argument("--serve-prec", default="fp32", choices=sorted(PREC_NAMES))
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-small-arena-gb", type=float, default=8.0)
    ap.add_argument("--serve-pack", type=int, default=8,
                    help="largest packed group of small serving requests (1: no packing)")
    ap.add_argument("--serve-only", action="store_true",
                    help="print the serving measurement as the JSON line (no residual timing)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, used to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); a multi-GPU run would "
              "shard the triple loop by triples with one all-reduce of the residual, and is not "
              "implemented.", file=sys.stderr)
        return 2

    if args.serve_molecules > 0 and "GPU_MAX_HW_QUEUES" not in os.environ:
        # every serving slot uses two streams and the server one more for its copies;
        # streams beyond the runtime's hardware-queue count would wait on each other
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, 2 * args.serve_slots + 4))
    import torch

    from paper_2007_01088_amd import cc3
    from paper_2007_01088_amd.synth import make_inputs

    if args.serve_only:
        res = serve(args.serve_molecules, args.serve_calls, args.serve_prec, args.serve_slots,
                    args.serve_load, args.serve_small_arena_gb, max_pack=args.serve_pack)
        print(json.dumps({
            "metric": "Serving p50/p99 latency (ms) and aggregate TFLOP/s (4nv^4no^3/call)",
            "value": res["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": res["requests"],
            "warmup": 1, "ms_per_step": res["makespan_s"] * 1e3 / res["requests"],
            "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
            "dtype": res["prec"], "data": "synthetic (seeded Cholesky-factored molecules)",
            "config": {"workload": f"serving mix: {res['molecules']} molecules, no U[5,20], "
                                   f"nv U[60,250], nchol 3(no+nv), {res['calls_per_molecule']} "
                                   "closed-loop calls each, Poisson arrivals"},
            "serving": res}), flush=True)
        return 0

    no, nv, nchol = WORKLOADS[args.workload]
    log(f"workload {args.workload}: no={no} nv={nv} nchol={nchol} prec={args.prec}")
    d = make_inputs(no, nv, nchol)
    dev = torch.device("cuda:0")
    g = {k: torch.from_numpy(d[k]).to(dev) for k in ("eps", "L", "t1", "t2")}
    o1 = torch.empty((no, nv), dtype=torch.float64, device=dev)
    o2 = torch.empty((no, no, nv, nv), dtype=torch.float64, device=dev)
    ctx = cc3.Context(0)
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb << 17  # doubles
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n * 8} bytes read and {n * 8} bytes written")
        del src, dst
    for w in range(args.warmup):
        ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], o1, o2)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], o1, o2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = ctx.profile_get()
    ctx.profile_enable(False)
    log(f"timed {args.steps} steps in {dt:.3f} s")
    nominal, executed = cc3.flops(no, nv)
    ms = dt / args.steps * 1e3
    value = nominal / (dt / args.steps) / 1e12
    nx = max(1, args.extra_steps)

    dom = max((k for k in stats if k in DOMINANT_SOURCES), key=lambda k: stats[k]["total_ms"])
    st = stats[dom]
    avg_ms = st["total_ms"] / st["launches"]
    flops_per_launch = st["flops"] / st["launches"]
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS["fp64"]
    roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(dom, args.workload),
            "kernel": dom, "avg_launch_ms": avg_ms, "flops_per_launch": flops_per_launch}
    kernels = {k: {"launches": v["launches"], "avg_ms": v["total_ms"] / v["launches"],
                   "share": v["total_ms"] / max(1e-9, sum(x["total_ms"] for x in stats.values()))}
               for k, v in stats.items()}
    # Two-stream overlap of consecutive batches stretches each launch in the timed
    # region; the same call with CC3_ONE_STREAM (after it, untimed for `value`) gives
    # every kernel's duration without a neighbour on the device.
    standalone = None
    if args.standalone_steps > 0:
        ctx.profile_enable(True)
        for _ in range(args.standalone_steps):
            ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], o1, o2, flags=cc3.ONE_STREAM)
        torch.cuda.synchronize()
        st_s = ctx.profile_get()
        ctx.profile_enable(False)
        s_dom = st_s[dom]
        s_avg = s_dom["total_ms"] / s_dom["launches"]
        s_ach = (s_dom["flops"] / s_dom["launches"]) / (s_avg * 1e-3) / 1e12
        standalone = {
            "steps": args.standalone_steps,
            "roofline": {"bound": "mfma", "achieved": s_ach, "peak": peak, "unit": "TFLOP/s",
                         "frac": s_ach / peak, "kernel": dom, "avg_launch_ms": s_avg},
            "kernels": {k: {"launches": v["launches"], "avg_ms": v["total_ms"] / v["launches"],
                            "tflops": (v["flops"] / v["total_ms"] * 1e-9) if v["flops"] else None}
                        for k, v in st_s.items()},
        }
        roof["standalone_frac"] = s_ach / peak
        roof["standalone_avg_launch_ms"] = s_avg
        log(f"standalone {dom}: {s_avg:.3f} ms per launch, {s_ach:.1f} TFLOP/s "
            f"({100 * s_ach / peak:.0f}% of peak)")
    # one sampled parity check of the timed output against nothing else than its own symmetry
    sym = float((o2 - o2.permute(1, 0, 3, 2)).abs().max() / o2.abs().max())

    mixed = {}
    if not args.no_mixed:
        # the same call with the W contractions in low precision; errors against the FP64
        # result of this GPU (equal to the CPU oracle to ~1e-15 in the parity tests)
        forms = set(args.mixed_forms.split(","))
        for name, prec in (("fp32", cc3.FP32), ("bf16x6", cc3.BF16X6), ("bf16x3", cc3.BF16X3)):
            if name not in forms:
                continue
            m1 = torch.empty_like(o1)
            m2 = torch.empty_like(o2)
            ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], m1, m2, prec=prec)
            torch.cuda.synchronize()
            log(f"mixed {name}: untimed call done")
            ctx.profile_enable(True)
            t0 = time.perf_counter()
            for _ in range(nx):
                ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], m1, m2, prec=prec)
            torch.cuda.synchronize()
            dtm = (time.perf_counter() - t0) / nx
            st_m = ctx.profile_get()
            ctx.profile_enable(False)
            w = st_m.get("w_build", {"total_ms": 0.0, "launches": 1, "flops": 0.0})
            mixed[name] = {
                "value": nominal / dtm / 1e12, "ms_per_step": dtm * 1e3,
                "rel_err_omega1": float((m1 - o1).norm() / o1.norm()),
                "rel_err_omega2": float((m2 - o2).norm() / o2.norm()),
                "w_build_tflops": w["flops"] / (w["total_ms"] * 1e-3) / 1e12 if w["total_ms"] else None,
                "peak_tflops": PEAK_TFLOPS["fp32"] if name == "fp32" else PEAK_TFLOPS["bf16"] /
                (3 if name == "bf16x3" else 6),
            }
            log(f"mixed {name}: {mixed[name]['value']:.2f} TFLOP/s, "
                f"err {mixed[name]['rel_err_omega1']:.2e}/{mixed[name]['rel_err_omega2']:.2e}")
        # "mixed-all": the vv and Omega1 contraction in the low precision as well
        for name, prec in (("fp32_all", cc3.FP32), ("bf16x6_all", cc3.BF16X6),
                           ("bf16x3_all", cc3.BF16X3)):
            if name not in forms:
                continue
            m1 = torch.empty_like(o1)
            m2 = torch.empty_like(o2)
            fl = cc3.LOWP_CONTRACT
            ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], m1, m2, prec=prec, flags=fl)
            torch.cuda.synchronize()
            log(f"mixed {name}: untimed call done")
            ctx.profile_enable(True)
            t0 = time.perf_counter()
            for _ in range(nx):
                ctx.triples_residual(g["eps"], g["L"], g["t1"], g["t2"], m1, m2, prec=prec, flags=fl)
            torch.cuda.synchronize()
            dtm = (time.perf_counter() - t0) / nx
            st_m = ctx.profile_get()
            ctx.profile_enable(False)
            om = st_m.get("omega_contract", {"total_ms": 0.0, "launches": 1, "flops": 0.0})
            mixed[name] = {
                "value": nominal / dtm / 1e12, "ms_per_step": dtm * 1e3,
                "rel_err_omega1": float((m1 - o1).norm() / o1.norm()),
                "rel_err_omega2": float((m2 - o2).norm() / o2.norm()),
                "omega_contract_tflops": om["flops"] / (om["total_ms"] * 1e-3) / 1e12
                if om["total_ms"] else None,
                "what": "W and the vv/Omega1 contraction in this precision (CC3_LOWP_CONTRACT); "
                        "oo, Fock and back-transformation FP64",
            }
            log(f"mixed {name}: {mixed[name]['value']:.2f} TFLOP/s, "
                f"err {mixed[name]['rel_err_omega1']:.2e}/{mixed[name]['rel_err_omega2']:.2e}")

    out = {
        "metric": "Triples-residual TFLOP/s (4nv^4no^3/call)",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Cholesky-factored integrals, t1, t2)",
        "config": {"workload": f"CC3 triples residual no={no} nv={nv} nchol={nchol}",
                   "no": no, "nv": nv, "nchol": nchol, "prec": args.prec,
                   "nominal_flop_per_call": nominal, "executed_flop_per_call": executed},
        "roofline": roof,
        "kernels": kernels,
        "standalone": standalone,
        "omega2_pair_symmetry": sym,
    }
    if mixed:
        out["mixed"] = mixed
    if not args.no_jacobian_prep:
        # Algorithm 2 (the t3-dependent intermediates of the Jacobian preparation) on the
        # same inputs; nominal cost as one ground-state call, 4 nv^4 no^3
        zv = torch.empty((nv, nv, no, nv), dtype=torch.float64, device=dev)
        zo = torch.empty((nv, no, no, no), dtype=torch.float64, device=dev)
        ctx.jacobian_prep(g["eps"], g["L"], g["t1"], g["t2"], zv, zo)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(nx):
            ctx.jacobian_prep(g["eps"], g["L"], g["t1"], g["t2"], zv, zo)
        torch.cuda.synchronize()
        dtj = (time.perf_counter() - t0) / nx
        stj = ctx.profile_get()
        ctx.profile_enable(False)
        out["jacobian_prep"] = {
            "what": "Z~v_{abid} and Z~o_{ajil} of the preparation for the Jacobian transformations",
            "value": nominal / dtj / 1e12, "unit": "TFLOP/s", "ms_per_step": dtj * 1e3,
            "kernels": {k: {"launches": v["launches"], "avg_ms": v["total_ms"] / v["launches"],
                            "tflops": (v["flops"] / (v["total_ms"] * 1e-3) / 1e12)
                            if v["flops"] and v["total_ms"] else None}
                        for k, v in stj.items()},
        }
        log(f"jacobian prep: {out['jacobian_prep']['value']:.2f} TFLOP/s, {dtj * 1e3:.1f} ms per call")
        del zv, zo
    if not args.no_density:
        # Algorithm 3 (the triples contributions to the transition densities, FP64) for a
        # seeded left state on the same inputs; nominal cost 13 nv^4 no^3, the paper's count
        # for its occupied plus virtual loops; one untimed and one timed call
        from paper_2007_01088_amd.synth import make_left_inputs
        lf = make_left_inputs(no, nv)
        l1 = torch.from_numpy(lf["l1"]).to(dev)
        l2 = torch.from_numpy(lf["l2"]).to(dev)
        dens = ctx.transition_density(g["eps"], g["L"], g["t1"], g["t2"], l1, l2, lf["omega"])
        torch.cuda.synchronize()
        log("transition density: untimed call done")
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        ctx.transition_density(g["eps"], g["L"], g["t1"], g["t2"], l1, l2, lf["omega"], out=dens + (None,))
        torch.cuda.synchronize()
        dtd = time.perf_counter() - t0
        std = ctx.profile_get()
        ctx.profile_enable(False)
        nominal_d = 13.0 * nv ** 4 * no ** 3
        fams = {k: {"launches": v["launches"], "avg_ms": v["total_ms"] / v["launches"],
                    "tflops": (v["flops"] / (v["total_ms"] * 1e-3) / 1e12)
                    if v["flops"] and v["total_ms"] else None}
                for k, v in std.items()}
        ddom = max((k for k in std if std[k]["flops"]), key=lambda k: std[k]["total_ms"])
        dach = fams[ddom]["tflops"]
        out["transition_density"] = {
            "what": "Algorithm 3: D_cd, D_kc, D_ld, D_lk (FP64) for a seeded left state",
            "value": nominal_d / dtd / 1e12, "unit": "TFLOP/s", "ms_per_call": dtd * 1e3,
            "nominal_flop_per_call": nominal_d,
            "roofline": {"bound": "mfma", "kernel": ddom, "achieved": dach, "peak": PEAK_TFLOPS["fp64"],
                         "unit": "TFLOP/s", "frac": dach / PEAK_TFLOPS["fp64"]},
            "kernels": fams,
        }
        log(f"transition density: {out['transition_density']['value']:.2f} TFLOP/s, "
            f"{dtd * 1e3:.1f} ms per call")
        del dens, l1, l2
    if not args.no_cvs:
        # the core-valence separation worklist: only the triples that contain the lowest
        # occupied orbital (one core orbital of interest), through the subset entry point
        core = cc3.cvs_triples(no, [0])
        ctx.triples_residual_subset(g["eps"], g["L"], g["t1"], g["t2"], core)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nx):
            ctx.triples_residual_subset(g["eps"], g["L"], g["t1"], g["t2"], core)
        torch.cuda.synchronize()
        dtc = (time.perf_counter() - t0) / nx
        ntri = len(cc3.cvs_triples(no, list(range(no))))
        out["cvs"] = {"what": "contravariant residual over the CVS worklist (triples with "
                              "occupied orbital 0 as the core index), cc3_triples_residual_subset",
                      "core": [0], "triples": int(len(core)), "of_triples": int(ntri),
                      "ms_per_call": dtc * 1e3, "full_call_ms": ms, "speedup": ms / (dtc * 1e3)}
        log(f"cvs worklist: {len(core)} of {ntri} triples, {dtc * 1e3:.1f} ms per call "
            f"({ms / (dtc * 1e3):.1f}x faster than the full call)")
    if not args.no_host_buffers:
        # the same call with every array in pinned host memory: the PCIe-inclusive rate
        # (inputs staged into the workspace, outputs copied back, the call waits)
        h = {k: v.cpu().pin_memory() for k, v in g.items()}
        h1 = torch.empty((no, nv), dtype=torch.float64).pin_memory()
        h2 = torch.empty((no, no, nv, nv), dtype=torch.float64).pin_memory()
        ctx.triples_residual(h["eps"], h["L"], h["t1"], h["t2"], h1, h2)
        t0 = time.perf_counter()
        for _ in range(nx):
            ctx.triples_residual(h["eps"], h["L"], h["t1"], h["t2"], h1, h2)
        dth = (time.perf_counter() - t0) / nx
        same = bool(torch.equal(h2, o2.cpu()) and torch.equal(h1, o1.cpu()))
        in_bytes = sum(v.numel() * 8 for v in h.values())
        out["host_buffers"] = {
            "what": "cc3_triples_residual with inputs and outputs in pinned host memory "
                    "(PCIe transfers inside the timed call)",
            "value": nominal / dth / 1e12, "unit": "TFLOP/s", "ms_per_call": dth * 1e3,
            "bytes_in": in_bytes, "bytes_out": (h1.numel() + h2.numel()) * 8,
            "equal_to_device_call": same}
        log(f"host buffers: {dth * 1e3:.1f} ms per call ({nominal / dth / 1e12:.2f} TFLOP/s), "
            f"bit-equal to the device call: {same}")
        del h, h1, h2
    if args.serve_molecules > 0:
        ctx.close()
        del g, o1, o2
        torch.cuda.empty_cache()
        out["serving"] = serve(args.serve_molecules, args.serve_calls, args.serve_prec,
                               args.serve_slots, args.serve_load, args.serve_small_arena_gb,
                               max_pack=args.serve_pack)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(no, nv, nchol, args.cpu_budget)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
