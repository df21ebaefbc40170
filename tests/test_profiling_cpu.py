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


def test_mfma_summary_busy_share_and_rate(tmp_path):
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration integer)")
    con.executemany("insert into kernels values (?, ?)",
                    [("cc3::k_wbuild<0>(x)", 2_000_000), ("cc3::k_wbuild<0>(x)", 2_000_000),
                     ("cc3::k_mix<512>(y)", 500_000)])
    con.commit()
    con.close()
    fields = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    pmc = tmp_path / "m.csv"
    with open(pmc, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for disp in (1, 2):
            for c, v in (("SQ_VALU_MFMA_BUSY_CYCLES", 512.0e6), ("GRBM_GUI_ACTIVE", 8.0e6),
                         ("SQ_INSTS_VALU_MFMA_MOPS_F64", 1.0e11 / 512)):
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": "cc3::k_wbuild<0>(x)",
                            "Counter_Name": c, "Counter_Value": v})
        w.writerow({"Dispatch_Id": 3, "Kernel_Name": "cc3::k_mix<512>(y)",
                    "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": 1.0e5})
    rows = {r["kernel"]: r for r in P.mfma_summary(str(db), str(pmc), None, None, None, ".", None)}
    wb = rows["cc3::k_wbuild<0>"]
    # GRBM_GUI_ACTIVE is summed over the 8 XCDs: 512e6 busy cycles over 1e6 chip cycles
    # x 1024 SIMDs is half the SIMD cycles
    assert wb["mfma_busy"] == pytest.approx(0.5)
    # 1e11 FLOP in 2 ms: 50 TFLOP/s, of the 78.6 TFLOP/s FP64 peak
    assert wb["mfma_type"] == "F64" and wb["mfma_tflops"] == pytest.approx(50.0)
    assert wb["peak_frac"] == pytest.approx(50.0 / 78.6)
    assert rows["cc3::k_mix<512>"]["mfma_type"] is None
    assert "`cc3::k_wbuild<0>`" in P.mfma_markdown(list(rows.values()), "cmd")
