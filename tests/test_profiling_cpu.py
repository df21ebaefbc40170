"""Host-side summaries of rocprofv3 output (paper_2007_01088_amd/profiling.py) on
small synthetic files: per-kernel statistics and calibrated HBM traffic."""
import csv
import sqlite3

import pytest

from paper_2007_01088_amd import profiling as P


def test_kernel_stats_groups_by_kernel(tmp_path):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer)")
    rows = [("void cc3::k_omega<2>(double const*, int)", 4000), ("cc3::k_omega<2>(x)", 6000),
            ("cc3::k_mix(double const*)", 1000)]
    con.executemany("insert into kernels values (?, ?)", rows)
    con.commit()
    con.close()
    st = {r["kernel"]: r for r in P.kernel_stats(str(db))}
    assert st["cc3::k_omega<2>"]["launches"] == 2
    assert st["cc3::k_omega<2>"]["avg_us"] == pytest.approx(5.0)
    assert st["cc3::k_mix"]["share"] == pytest.approx(1000 / 11000)
    md = P.stats_markdown(list(st.values()), "cmd")
    assert "`cc3::k_mix`" in md and "cmd" in md


def _write_counters(path, counter, entries):
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for disp, name, val in entries:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": val})


def test_traffic_scales_by_copy_calibration(tmp_path):
    gib = 1 << 30
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    # the copy of 1 GiB reads as half on FETCH_SIZE and whole on WRITE_SIZE (KiB)
    _write_counters(fetch, "FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", gib / 2048),
                                          (2, "cc3::k_omega<1>(a)", 100.0),
                                          (3, "cc3::k_omega<1>(a)", 300.0)])
    _write_counters(write, "WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", gib / 1024),
                                          (2, "cc3::k_omega<1>(a)", 50.0),
                                          (3, "cc3::k_omega<1>(a)", 50.0)])
    r = P.traffic(str(fetch), str(write), "k_omega", float(gib))
    assert r["dispatches"] == 2
    assert r["calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert r["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)
    assert r["write_bytes_per_launch"] == pytest.approx(50.0 * 1024)
    r0 = P.traffic(str(fetch), str(write), "k_omega", None)
    assert r0["calibration"] is None and r0["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024)
