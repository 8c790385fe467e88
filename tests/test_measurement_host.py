"""Host logic of the measurements that bench.py reports: the rocprofv3
counter summaries (calibrated HBM traffic, VALU flop rates and issue
fraction) on synthetic counter files whose answers are known by hand, the
algorithmic-bytes formula on a tiny system, and the refusal of a traffic
record taken from other kernel sources or another launch tuning."""
import csv
import json
import os

import pytest

from paper_2503_13075_amd import rocprof_summary as R

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (kernel, name, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": name, "Counter_Value": value})


def test_traffic_is_calibrated_by_the_copy_and_summed_over_solve_kernels(tmp_path):
    mib = 4
    copy_bytes = mib << 20
    fetch, write = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the copy reads copy_bytes but FETCH_SIZE reports half of it (in KiB),
    # WRITE_SIZE reports it exactly; two solves of two solve-kernel dispatches
    _write(fetch, [("__amd_rocclr_copyBuffer", "FETCH_SIZE", copy_bytes / 2 / 1024),
                   ("void solve_kernel<float, unsigned short, 0, 512, false, 2>(...)", "FETCH_SIZE", 1000.0),
                   ("reset_counters", "FETCH_SIZE", 24.0),
                   ("void solve_kernel<float, unsigned short, 0, 512, false, 2>(...)", "FETCH_SIZE", 1000.0),
                   ("reset_counters", "FETCH_SIZE", 24.0),
                   ("some_other_kernel", "FETCH_SIZE", 1e9)])
    _write(write, [("__amd_rocclr_copyBuffer", "WRITE_SIZE", copy_bytes / 1024),
                   ("void solve_kernel<double, unsigned short, 0, 128, false, 2>(...)", "WRITE_SIZE", 300.0),
                   ("void solve_kernel<double, unsigned short, 0, 128, false, 2>(...)", "WRITE_SIZE", 300.0)])
    res = R.traffic(fetch, write, 2, mib, 1.0e6)
    assert res["fetch_calibration_factor"] == pytest.approx(2.0)
    assert res["write_calibration_factor"] == pytest.approx(1.0)
    assert res["raw_fetch_kib_per_solve"] == pytest.approx(1024.0)
    assert res["fetch_bytes_per_solve"] == pytest.approx(1024.0 * 1024.0 * 2.0)
    assert res["write_bytes_per_solve"] == pytest.approx(300.0 * 1024.0)
    assert res["traffic_over_algorithmic"] == pytest.approx((2 * 1024.0 * 1024.0 + 300.0 * 1024.0) / 1.0e6)


def test_valu_rates_and_issue_fraction(tmp_path):
    d1, d2 = str(tmp_path / "p1"), str(tmp_path / "p2")
    k = "void solve_kernel<float, unsigned short, 0, 512, false, 4>(...)"
    # per solve (2 solves): 100 FP64 adds, 50 muls, 10 transcendentals, 20 fmas;
    # 1,000 VALU instructions in all
    _write(d1, [(k, "SQ_INSTS_VALU_ADD_F64", 200.0), (k, "SQ_INSTS_VALU_MUL_F64", 100.0),
                (k, "SQ_INSTS_VALU_TRANS_F64", 20.0), (k, "SQ_INSTS_VALU_FMA_F64", 40.0),
                (k, "SQ_INSTS_VALU_ADD_F32", 0.0), (k, "SQ_INSTS_VALU_MUL_F32", 0.0),
                (k, "SQ_INSTS_VALU_TRANS_F32", 0.0), (k, "SQ_INSTS_VALU_FMA_F32", 2.0),
                ("__amd_rocclr_copyBuffer", "SQ_INSTS_VALU_ADD_F64", 1e9)])
    _write(d2, [(k, "SQ_INSTS_VALU", 2000.0)])
    ms = 0.5
    res = R.valu([d1, d2], 2, ms)
    f64 = 64.0 * (100 + 50 + 10 + 2 * 20)
    assert res["f64_flops_per_solve"] == pytest.approx(f64)
    assert res["f64_tflops"] == pytest.approx(f64 / (ms / 1e3) / 1e12)
    assert res["f64_frac_of_peak"] == pytest.approx(f64 / (ms / 1e3) / 1e12 / R.PEAK_F64_VEC_TFLOPS)
    assert res["f32_flops_per_solve"] == pytest.approx(64.0 * 2 * 1)
    assert res["valu_issue_fraction"] == pytest.approx(1000.0 * 4 / (R.N_SIMD * R.CLOCK_HZ * ms / 1e3))


def test_algorithmic_bytes_formula():
    import bench
    # 3 atoms, 2 constraints, L with one off-diagonal entry: factor_entries
    # counts the n diagonal entries and both triangles
    st = {"atoms": 3, "constraints": 2, "factor_entries": 2 + 2 * 1}
    assert bench.algorithmic_bytes(None, st) == 80 * 3 + 24 * 2 + 4 * 1 + 8 * 2


def test_traffic_record_is_refused_when_stale(tmp_path, monkeypatch):
    import bench
    from paper_2503_13075_amd.build import kernel_source_hash
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tuning = {"band_block": [1024, 128, 512, 512, 1024], "lds_limit": 0}
    rec = {"traffic_bytes_per_solve": 123.0, "kernel_source_sha256_16": kernel_source_hash(),
           "tuning": tuning, "variant": "decoupled"}
    path = prof / "solve_kernel_tiny_traffic.json"
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("tiny", "decoupled", tuning) == 123.0
    assert bench.measured_traffic("tiny", "mixed", tuning) is None                     # other variant
    assert bench.measured_traffic("tiny", "decoupled", dict(tuning, lds_limit=1)) is None  # other tuning
    path.write_text(json.dumps(dict(rec, kernel_source_sha256_16="0" * 16)))
    assert bench.measured_traffic("tiny", "decoupled", tuning) is None                 # other sources
    assert bench.measured_traffic("absent", "decoupled", tuning) is None
