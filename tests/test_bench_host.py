"""Host logic of the benchmark (CPU only): the one-GPU guard and the HBM
traffic summary built from rocprofv3 counter files."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

GIB = float(1 << 30)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "123_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for d, name, v in rows:
            w.writerow([d, name, counter, v])


@pytest.fixture
def counter_runs(tmp_path):
    fp64 = "void rtbte::k_items<16, true, false, false>(rtbte::RowArgs)"
    plain = "void rtbte::k_items<16, false, false, false>(rtbte::RowArgs)"
    deriv = "void rtbte::k_items<16, true, true, false>(rtbte::RowArgs)"   # rates: not a benchmark kernel
    mixed = "void rtbte::k_items_mixed<16, true, false>(rtbte::MixArgs)"
    copy = "__amd_rocclr_copyBuffer"
    # the calibration copy comes first; a later 4 GiB copy reads four times as much
    fetch = [(1, copy, 524288.0), (2, fp64, 3.0e6), (3, fp64, 3.2e6), (4, plain, 4.0e6), (5, deriv, 9e9),
             (6, mixed, 2.0e6), (7, copy, 4 * 524288.0)]
    write = [(1, copy, 1048576.0), (2, fp64, 5000.0), (3, fp64, 5000.0), (4, plain, 5000.0), (5, deriv, 7.0),
             (6, mixed, 5000.0), (7, copy, 4 * 1048576.0)]
    _counter_csv(str(tmp_path / "fetch" / "host"), "FETCH_SIZE", fetch)
    _counter_csv(str(tmp_path / "write" / "host"), "WRITE_SIZE", write)
    rec = {"config": {"workload": "unit"}, "roofline": {"algorithmic_bytes_per_launch": 6.0e9},
           "fp64_plain_channels": {"roofline": {"algorithmic_bytes_per_launch": 8.0e9}},
           "mixed": {"roofline": {"algorithmic_bytes_per_launch": 4.0e9}}}
    with open(tmp_path / "fetch.json", "w") as f:
        f.write("a line of other output\n" + json.dumps(rec) + "\n")
    return tmp_path


def test_traffic_summary(counter_runs, capsys):
    import bench
    out = counter_runs / "traffic.json"
    bench.traffic_summary(str(counter_runs / "fetch"), str(counter_runs / "write"),
                          str(counter_runs / "fetch.json"), "unit", out_path=str(out))
    d = json.loads(out.read_text())
    assert d["fetch_scale"] == pytest.approx(2.0) and d["write_scale"] == pytest.approx(1.0)
    e = d["fp64"]
    assert e["kernel"] == "void rtbte::k_items<16, true, false, false>" and e["dispatches"] == 2
    hbm = (3.1e6 * 2.0 + 5000.0) * 1024
    assert e["hbm_bytes_per_launch"] == pytest.approx(hbm)
    assert e["ratio"] == pytest.approx(hbm / 6.0e9)
    assert e["kernel_source_hash"] == bench.kernel_source_hash()
    assert d["fp64_plain"]["ratio"] == pytest.approx((4.0e6 * 2 + 5000.0) * 1024 / 8.0e9)
    assert d["mixed"]["ratio"] == pytest.approx((2.0e6 * 2 + 5000.0) * 1024 / 4.0e9)
    assert all("rocprofv3 --pmc" in c for c in d["commands"][:2])


def test_valu_summary(tmp_path):
    """The ph-ph-only launches (fewest instructions) of the matrix-free FP64
    kernel give the instructions per stored ph-ph channel."""
    import bench
    mf = "void rtbte::k_items<16, true, false, true>(rtbte::RowArgs)"
    mf_mixed = "void rtbte::k_items_mixed<16, true, true>(rtbte::MixArgs)"
    stored = "void rtbte::k_items<16, true, false, false>(rtbte::RowArgs)"
    rows = [(1, stored, 3.6e8), (2, mf, 2.0e9), (3, mf, 2.0e9), (4, mf, 2.3e9), (5, mf, 2.3e9),
            (6, mf_mixed, 1.0e9)]
    _counter_csv(str(tmp_path / "valu" / "host"), "SQ_INSTS_VALU", rows)
    rec = {"config": {"workload": "unit", "stored_channels": [10, 20, 3.2e8]}}
    with open(tmp_path / "valu.json", "w") as f:
        f.write(json.dumps(rec) + "\n")
    out = tmp_path / "valu_out.json"
    bench.valu_summary(str(tmp_path / "valu"), str(tmp_path / "valu.json"), "unit", out_path=str(out))
    d = json.loads(out.read_text())
    assert d["dispatches"] == 4 and d["kernel"] == "void rtbte::k_items<16, true, false, true>"
    assert d["lane_instructions_per_channel"] == pytest.approx(2.0e9 * 64 / 3.2e8)
    assert d["kernel_source_hash"] == bench.kernel_source_hash()
