"""Summaries of rocprofv3 output for the kernels of libcc3 (host-side tooling).

    python -m paper_2007_01088_amd.profiling stats RUN_results.db [--out FILE.md] [--cmd "..."]
        per-kernel launches, average and total duration from a --kernel-trace database
    python -m paper_2007_01088_amd.profiling traffic --fetch F.csv --write W.csv --kernel REGEX
        [--calib-bytes N] [--source-sha SHA] [--out FILE.json] [--cmd "..."]
        HBM bytes per dispatch from two --pmc runs (FETCH_SIZE, WRITE_SIZE, in KiB),
        scaled by what the same counters read for the device-to-device copy of a
        known size (the largest __amd_rocclr_copyBuffer dispatch) when N is given
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import re
import sqlite3
import sys


def _short(name: str) -> str:
    return re.sub(r"\(.*", "", name).replace("void ", "").strip()


def kernel_stats(db_path: str) -> list[dict]:
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, duration from kernels").fetchall()
    con.close()
    agg = collections.OrderedDict()
    for name, dur in rows:
        k = _short(name)
        a = agg.setdefault(k, [0, 0.0])
        a[0] += 1
        a[1] += dur
    total = sum(a[1] for a in agg.values()) or 1.0
    out = [{"kernel": k, "launches": n, "avg_us": t / n / 1e3, "total_ms": t / 1e6,
            "share": t / total} for k, (n, t) in agg.items()]
    out.sort(key=lambda r: -r["total_ms"])
    return out


def stats_markdown(rows: list[dict], cmd: str | None) -> str:
    lines = []
    if cmd:
        lines += ["Command:", "", "    " + cmd, ""]
    lines += ["| kernel | launches | avg (us) | total (ms) | share |", "|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['kernel']}` | {r['launches']} | {r['avg_us']:.1f} | "
                     f"{r['total_ms']:.2f} | {100 * r['share']:.1f}% |")
    return "\n".join(lines) + "\n"


def _counter(csv_path: str, counter: str) -> dict:
    """{kernel short name: [per-dispatch values]} for one counter."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            per[_short(r["Kernel_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def traffic(fetch_csv: str, write_csv: str, kernel_re: str, calib_bytes: float | None) -> dict:
    fetch = _counter(fetch_csv, "FETCH_SIZE")
    write = _counter(write_csv, "WRITE_SIZE")
    pat = re.compile(kernel_re)
    names = [k for k in fetch if pat.search(k)]
    if not names:
        raise SystemExit(f"no kernel matching {kernel_re!r} in {fetch_csv}")
    fvals = [v for k in names for v in fetch[k]]
    wvals = [v for k in names for v in write.get(k, [])]
    f_kib = sum(fvals) / len(fvals)
    w_kib = sum(wvals) / len(wvals) if wvals else 0.0
    scale_f = scale_w = 1.0
    calib = None
    if calib_bytes:
        cf = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
        cw = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
        if cf > 0 and cw > 0:
            scale_f = calib_bytes / (cf * 1024.0)
            scale_w = calib_bytes / (cw * 1024.0)
            calib = {"copy_bytes": calib_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
                     "fetch_scale": scale_f, "write_scale": scale_w}
    fb = f_kib * 1024.0 * scale_f
    wb = w_kib * 1024.0 * scale_w
    return {"kernels": names, "dispatches": len(fvals), "fetch_bytes_per_launch": fb,
            "write_bytes_per_launch": wb, "hbm_bytes_per_launch": fb + wb, "calibration": calib}


def _per_dispatch(csv_path: str) -> dict:
    """{kernel short name: {dispatch id: {counter: value}}} from a --pmc CSV."""
    per = collections.defaultdict(lambda: collections.defaultdict(dict))
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            d = per[_short(r["Kernel_Name"])][r["Dispatch_Id"]]
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return per


PEAKS = {"F64": 78.6, "F32": 157.3, "BF16": 2516.6}


def mfma_summary(trace_db: str, mfma_csv: str, fetch_csv: str | None, write_csv: str | None,
                 lds_csv: str | None, kernel_re: str, calib_bytes: float | None,
                 simds: int = 1024, xcds: int = 8) -> list[dict]:
    """Per kernel: average duration (kernel trace), MFMA busy share of the SIMD cycles
    (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs x SIMDs)), FLOP counted by the
    MFMA units (SQ_INSTS_VALU_MFMA_MOPS_* x 512) and their rate, HBM bytes per dispatch
    (calibrated FETCH_SIZE / WRITE_SIZE), the LDS bank-conflict share of the LDS-active
    cycles and the share of wave cycles spent waiting on LDS instructions.

    rocprofv3 reports GRBM_GUI_ACTIVE summed over the XCDs: a fill kernel of 164.6 us
    reads 3.22e6 cycles, 8 x 2.44 GHz x its duration, so the per-XCD (chip) cycle count
    is GRBM_GUI_ACTIVE / 8 on MI355X."""
    dur = {r["kernel"]: r for r in kernel_stats(trace_db)}
    mf = _per_dispatch(mfma_csv)
    tr = {}
    if fetch_csv and write_csv:
        fetch = _counter(fetch_csv, "FETCH_SIZE")
        write = _counter(write_csv, "WRITE_SIZE")
        sf = sw = 1.0
        if calib_bytes:
            cf = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
            cw = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
            if cf > 0 and cw > 0:
                sf, sw = calib_bytes / (cf * 1024.0), calib_bytes / (cw * 1024.0)
        for k in fetch:
            fv, wv = fetch[k], write.get(k, [])
            tr[k] = (sum(fv) / len(fv) * 1024 * sf, (sum(wv) / len(wv) * 1024 * sw) if wv else 0.0)
    lds = _per_dispatch(lds_csv) if lds_csv else {}
    pat = re.compile(kernel_re)
    out = []
    for k, disp in mf.items():
        if not pat.search(k):
            continue
        n = len(disp)
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in disp.values())
        gui = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in disp.values())
        flops = {t: sum(d.get(f"SQ_INSTS_VALU_MFMA_MOPS_{t}", 0.0) for d in disp.values()) * 512 / n
                 for t in PEAKS}
        kind = max(flops, key=lambda t: flops[t])
        avg_us = dur[k]["avg_us"] if k in dur else None
        rate = flops[kind] / (avg_us * 1e-6) / 1e12 if avg_us and flops[kind] else None
        row = {"kernel": k, "dispatches": n, "avg_us": avg_us,
               "mfma_busy": busy / (gui / xcds * simds) if gui else None,
               "mfma_type": kind if flops[kind] else None,
               "mfma_flop_per_dispatch": flops[kind],
               "mfma_tflops": rate, "peak_frac": rate / PEAKS[kind] if rate else None}
        if k in tr:
            row["fetch_bytes"], row["write_bytes"] = tr[k]
        if k in lds:
            conf = sum(d.get("SQ_LDS_BANK_CONFLICT", 0.0) for d in lds[k].values())
            act = sum(d.get("SQ_LDS_IDX_ACTIVE", 0.0) for d in lds[k].values())
            row["lds_bank_conflict_share"] = conf / act if act else None
            wait = sum(d.get("SQ_WAIT_INST_LDS", 0.0) for d in lds[k].values())
            wave = sum(d.get("SQ_WAVE_CYCLES", 0.0) for d in lds[k].values())
            row["lds_wait_share"] = wait / wave if wave else None
        out.append(row)
    out.sort(key=lambda r: -(r["avg_us"] or 0) * r["dispatches"])
    return out


def mfma_markdown(rows: list[dict], cmd: str | None) -> str:
    lines = []
    if cmd:
        lines += ["Commands:", "", "    " + cmd, ""]
    lines += ["| kernel | dispatches | avg (us) | MFMA busy | MFMA FLOP / dispatch | counted TFLOP/s "
              "| of dtype peak | HBM read / written per dispatch | LDS bank conflicts | LDS wait |",
              "|---|---|---|---|---|---|---|---|---|---|"]
    for r in rows:
        def f(x, fmt):
            return format(x, fmt) if x is not None else "-"
        rb = (f"{r['fetch_bytes'] / 1e9:.3f} / {r['write_bytes'] / 1e9:.3f} GB"
              if "fetch_bytes" in r else "-")
        lines.append(
            f"| `{r['kernel']}` | {r['dispatches']} | {f(r['avg_us'], '.1f')} | "
            f"{f(r['mfma_busy'] * 100 if r['mfma_busy'] is not None else None, '.1f')}% | "
            f"{f(r['mfma_flop_per_dispatch'], '.3e')} {r['mfma_type'] or ''} | "
            f"{f(r['mfma_tflops'], '.1f')} | "
            f"{f(r['peak_frac'] * 100 if r['peak_frac'] else None, '.1f')}% | {rb} | "
            f"{f(r.get('lds_bank_conflict_share', None), '.3f')} | "
            f"{f(r.get('lds_wait_share', None), '.3f')} |")
    return "\n".join(lines) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2007_01088_amd.profiling")
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--out")
    s.add_argument("--cmd")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--calib-bytes", type=float)
    t.add_argument("--source-sha")
    t.add_argument("--out")
    t.add_argument("--cmd")
    m = sub.add_parser("mfma")
    m.add_argument("--trace", required=True, help="kernel-trace results database")
    m.add_argument("--mfma", required=True, help="--pmc CSV with the MFMA counters")
    m.add_argument("--fetch")
    m.add_argument("--write")
    m.add_argument("--lds")
    m.add_argument("--kernel", default=".")
    m.add_argument("--calib-bytes", type=float)
    m.add_argument("--out")
    m.add_argument("--cmd")
    args = ap.parse_args(argv)
    if args.cmd_name == "mfma":
        rows = mfma_summary(args.trace, args.mfma, args.fetch, args.write, args.lds, args.kernel,
                            args.calib_bytes)
        text = mfma_markdown(rows, args.cmd)
        if args.out:
            with open(args.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
        return 0
    if args.cmd_name == "stats":
        text = stats_markdown(kernel_stats(args.db), args.cmd)
        if args.out:
            with open(args.out, "w") as f:
                f.write(text)
        sys.stdout.write(text)
        return 0
    res = traffic(args.fetch, args.write, args.kernel, args.calib_bytes)
    if args.source_sha:
        res["source_sha"] = args.source_sha
    if args.cmd:
        res["commands"] = args.cmd
    text = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
