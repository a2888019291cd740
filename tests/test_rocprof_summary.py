"""Host logic of the profile summary (paper_2509_08383_amd/rocprof_summary.py) on small
synthetic rocprofv3 CSV files: the timed-CutMax window, the copy calibration of the byte
counters and the per-kernel aggregation."""
import csv
import os

import pytest

from paper_2509_08383_amd import rocprof_summary as rs


def _write(d, rows, counters=None):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_kernel_trace.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp",
                                          "Grid_Size_X", "Grid_Size_Y"])
        w.writeheader()
        for r in rows:
            w.writerow(r)
    if counters is not None:
        with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for c in counters:
                w.writerow(c)


def _trace(kernels):
    """dispatch rows: encryption, the kernels twice (warm-up, timed), decryption, a copy"""
    seq = ["k_encfinish(x)"] + kernels + kernels + ["k_decmul(x)", "k_copy(x)"]
    rows, t = [], 0
    for i, k in enumerate(seq):
        dur = 1000 * (i + 1)
        gx, gy = ("65536", "64") if k.startswith("k_copy") else ("256", "1")
        rows.append({"Dispatch_Id": i + 1, "Kernel_Name": k, "Start_Timestamp": t, "End_Timestamp": t + dur,
                     "Grid_Size_X": gx, "Grid_Size_Y": gy})
        t += dur + 10
    return rows


def test_window_calibration_and_aggregation(tmp_path):
    kernels = ["void he::k_ntt<4, 16, false, false, 0, 0>(he::VecSet)", "he::k_modup<10, 8>(a)",
               "void he::k_ntt<4, 16, false, false, 0, 0>(he::VecSet)"]
    rows = _trace(kernels)
    copy_id = rows[-1]["Dispatch_Id"]
    copy_bytes = 64 * 65536 * 8
    fetch = [{"Dispatch_Id": r["Dispatch_Id"], "Counter_Name": "FETCH_SIZE",
              "Counter_Value": (copy_bytes / 2 / 1024 if r["Dispatch_Id"] == copy_id else 100.0)} for r in rows]
    _write(str(tmp_path / "trace"), rows)
    _write(str(tmp_path / "fetch"), rows, fetch)
    s = rs.summarize(trace=str(tmp_path / "trace"), fetch=str(tmp_path / "fetch"))
    assert s["dispatches"] == 3                       # the timed half only
    assert abs(s["fetch_scale"] / 1024 - 2.0) < 1e-12  # the copy reads twice what FETCH_SIZE counts
    names = {e["kernel"]: e for e in s["kernels"]}
    assert set(names) == {"ntt_fwd_pass1", "k_modup"}
    assert names["ntt_fwd_pass1"]["launches"] == 2
    # timed half = dispatches 5, 6, 7: durations 5000, 6000, 7000 ns
    assert names["ntt_fwd_pass1"]["total_ms"] == pytest.approx((5000 + 7000) * 1e-6)
    assert names["k_modup"]["avg_us"] == pytest.approx(6.0)
    assert names["k_modup"]["fetch_MiB"] == pytest.approx(100.0 * 2048 / 2**20)
    assert "ntt_fwd_pass1" in rs.to_markdown(s)


def test_texture_unit_busy_fraction(tmp_path):
    rows = _trace(["he::k_inner_product_rot_lds<7, 3, 1>(a)"])
    # timed dispatch 3 lasts 3000 ns = 7200 cycles at 2.4 GHz on each of 256 CUs
    cyc = 256 * 3000e-9 * 2.4e9
    cnt = [{"Dispatch_Id": r["Dispatch_Id"], "Counter_Name": c, "Counter_Value": v * cyc}
           for r in rows for c, v in (("TA_TA_BUSY", 0.5), ("TD_TD_BUSY", 0.25))]
    _write(str(tmp_path / "tex"), rows, cnt)
    s = rs.summarize(tex=str(tmp_path / "tex"))
    (e,) = s["kernels"]
    assert e["kernel"] == "k_inner_product_rot"
    assert e["ta_busy"] == pytest.approx(0.5) and e["td_busy"] == pytest.approx(0.25)
    assert "ta_busy" in rs.to_markdown(s)


def test_per_launch_lists_the_timed_dispatches_of_a_class(tmp_path):
    rows = _trace(["void he::k_inner_product_rot_lds<7, 3, 1>(he::DevTables)", "he::k_modup<10, 8>(a)",
                   "void he::k_inner_product_rot<3, 7>(he::DevTables)"])
    _write(str(tmp_path / "trace"), rows)
    got = rs.per_launch(str(tmp_path / "trace"), "k_inner_product_rot")
    # the timed half: dispatches 5 and 7 (5000 and 7000 ns)
    assert [g[0] for g in got] == ["k_inner_product_rot_lds<7, 3, 1>", "k_inner_product_rot<3, 7>"]
    assert [g[2] for g in got] == [5.0, 7.0]


def test_mismatched_halves_are_rejected(tmp_path):
    rows = _trace(["he::k_modup<10, 8>(a)"])
    rows[2]["Kernel_Name"] = "he::k_tensor(a)"        # the timed half launches another kernel
    _write(str(tmp_path / "trace"), rows)
    with pytest.raises(RuntimeError):
        rs.summarize(trace=str(tmp_path / "trace"))


def test_kernel_class_names():
    assert rs.kernel_class("void he::k_ntt<4, 16, true, false, 0, 1>(he::VecSet)") == "ntt_fwd_pass2_moddown"
    assert rs.kernel_class("void he::k_ntt<4, 8, false, true, 0, 0>(x)") == "ntt_inv_pass1"
    assert rs.kernel_class("void he::k_ntt<3, 8, false, false, 1, 0>(x)") == "ntt_fwd_pass1_lift"
    assert rs.kernel_class("void he::k_ntt<4, 16, true, false, 0, 3, 0>(x)") == "ntt_fwd_pass2_moddown_rescale"
    assert rs.kernel_class("void he::k_ntt<4, 16, true, true, 0, 0, 1>(x)") == "ntt_inv_pass2_factored"
    assert rs.kernel_class("void he::k_ntt<4, 8, true, false, 0, 4, 0>(x)") == "ntt_fwd_pass2_moddown_chain"
    assert rs.kernel_class("void he::k_ntt<4, 16, true, true, 2, 0, 1>(x)") == "ntt_inv_pass2_tensor_factored"
    assert rs.kernel_class("void he::k_inner_product_rot<3>(he::DevTables)") == "k_inner_product_rot"
    assert rs.kernel_class("void he::k_inner_product_rot_reg<7, 3>(x)") == "k_inner_product_rot"
    assert rs.kernel_class("void he::k_inner_product_rot_lds<7, 3, 2>(x)") == "k_inner_product_rot"
