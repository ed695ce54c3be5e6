"""Host logic of the rocprofv3 summaries (synthetic CSV files)."""
import csv

from paper_2603_14040_amd import profiling as pf


def _write(path, rows, cols):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_kernel_stats(tmp_path):
    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [{"Kernel_Name": "void tph::(anonymous namespace)::k_a<float, 64>(int)", "Start_Timestamp": 0,
             "End_Timestamp": 10_000},
            {"Kernel_Name": "void tph::(anonymous namespace)::k_a<float, 64>(int)", "Start_Timestamp": 20_000,
             "End_Timestamp": 50_000},
            {"Kernel_Name": "k_b", "Start_Timestamp": 0, "End_Timestamp": 1_000}]
    _write(tmp_path / "run_kernel_trace.csv", rows, cols)
    st = pf.kernel_stats(str(tmp_path))
    assert st[0][0] == "k_a<f32,64>" and st[0][1] == 2 and abs(st[0][2] - 0.04) < 1e-12 and abs(st[0][3] - 20.0) < 1e-9
    assert st[1][0] == "k_b"


def test_traffic_calibrated_by_copy(tmp_path):
    cols = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    for sub, name, copyv, kv in (("f", "FETCH_SIZE", 512.0, 100.0), ("w", "WRITE_SIZE", 1024.0, 50.0)):
        d = tmp_path / sub
        d.mkdir()
        rows = [
            # the copy kernel of 1 MiB reads as 512 (fetch) / 1024 (write) KiB, split over two dimensions
            {"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 4096, "Counter_Name": name,
             "Counter_Value": copyv / 2},
            {"Dispatch_Id": 1, "Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 4096, "Counter_Name": name,
             "Counter_Value": copyv / 2},
            {"Dispatch_Id": 2, "Kernel_Name": "__amd_rocclr_copyBuffer", "Grid_Size": 64, "Counter_Name": name,
             "Counter_Value": 1.0},
            {"Dispatch_Id": 3, "Kernel_Name": "tph::k_smooth_tile<float>", "Grid_Size": 10, "Counter_Name": name,
             "Counter_Value": kv},
            {"Dispatch_Id": 4, "Kernel_Name": "tph::k_smooth_tile<float>", "Grid_Size": 10, "Counter_Name": name,
             "Counter_Value": 3 * kv},
            {"Dispatch_Id": 5, "Kernel_Name": "tph::k_other", "Grid_Size": 10, "Counter_Name": name,
             "Counter_Value": 1e6},
        ]
        _write(d / "run_counter_collection.csv", rows, cols)
    r = pf.traffic(str(tmp_path / "f"), str(tmp_path / "w"), r"k_smooth_tile<float", 1024 * 1024)
    # fetch: mean 200 KiB counted, calibration 1 MiB / 512 KiB = 2 -> 400 KiB; write: 100 KiB x 1 = 100 KiB
    assert r["fetch"]["launches"] == 2 and abs(r["fetch"]["calibration"] - 2.0) < 1e-12
    assert abs(r["fetch"]["bytes"] - 400 * 1024) < 1e-6 and abs(r["write"]["bytes"] - 100 * 1024) < 1e-6
    assert abs(r["bytes_per_launch"] - 500 * 1024) < 1e-6
    assert len(r["sources_sha256"]) == 64


def test_sources_hash_covers_the_smoother_files():
    import os
    csrc = os.path.join(os.path.dirname(pf.__file__), "csrc")
    for fn in pf.SMOOTHER_SOURCES:
        assert os.path.exists(os.path.join(csrc, fn))
    h = pf.sources_hash()
    assert len(h) == 64 and h == pf.sources_hash()
    assert pf.sources_hash(("common.h",)) != h
