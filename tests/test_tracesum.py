"""Host-only checks of the profile summarizer's counter mode (no device)."""
import csv

from paper_2005_06104_amd import tracesum


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_counters_window_average_and_calibration(tmp_path):
    k = "gemm_kernel<float, false, false, false, false, 1>(int)"
    rows = [
        (1, 1, k, "FETCH_SIZE", 999.0),                 # before the window: ignored
        (2, 2, "spin_kernel(long)", "FETCH_SIZE", 0.0),
        (3, 3, k, "FETCH_SIZE", 100.0),
        (3, 3, k, "FETCH_SIZE", 20.0),                  # a second dimension row of the same dispatch
        (4, 4, "other_kernel()", "FETCH_SIZE", 5.0),
        (5, 5, k, "FETCH_SIZE", 60.0),
        (6, 6, "spin_kernel(long)", "FETCH_SIZE", 0.0),
        (7, 7, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0),
    ]
    p = tmp_path / "counters.csv"
    _write(p, rows)
    out = tracesum.counters(str(p), "gemm_kernel<float", calib="copyBuffer", calib_bytes=1024 * 1024)
    assert out["dispatches"] == 2
    assert out["avg"]["FETCH_SIZE"] == 90.0
    # the 1 MiB copy reads 512 KiB by the counter: factor 2
    assert out["calib"]["factors"]["FETCH_SIZE"] == 2.0
    assert out["bytes_per_dispatch"]["FETCH_SIZE"] == 90.0 * 2.0 * 1024.0
