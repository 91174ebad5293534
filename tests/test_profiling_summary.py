"""The profiling summary's traffic arithmetic on synthetic rocprofv3 CSV files
(CPU only): counters scaled by what they read for a plain copy of known size,
and a calibration refused when the run holds other copies on the same grid."""
import csv
import os

import pytest

from paper_1805_10167_amd import profiling


def _write(path, rows, fields):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def _run(tmp_path, copy_fetch_kib):
    trace = [{"Kernel_Name": "hhg::k_x", "Grid_Size_X": 4096, "Start_Timestamp": 0, "End_Timestamp": 100000}]
    _write(str(tmp_path / "t" / "a_kernel_trace.csv"), trace,
           ["Kernel_Name", "Grid_Size_X", "Start_Timestamp", "End_Timestamp"])
    for tag, kern_kib, copies in (("f", 1000.0, copy_fetch_kib), ("w", 3000.0, [262144.0] * len(copy_fetch_kib))):
        rows = [{"Kernel_Name": "hhg::k_x", "Grid_Size": 4096, "Counter_Value": kern_kib}]
        rows += [{"Kernel_Name": profiling.COPY_KERNEL, "Grid_Size": 131072, "Counter_Value": c} for c in copies]
        _write(str(tmp_path / tag / "a_counter_collection.csv"), rows, ["Kernel_Name", "Grid_Size", "Counter_Value"])
    return profiling.summarize(str(tmp_path / "t"), str(tmp_path / "f"), str(tmp_path / "w"), "hhg::k_x",
                               268435456, "cmd")


def test_traffic_is_scaled_by_the_copy_calibration(tmp_path):
    # the copy of 256 MiB reads half its bytes on FETCH_SIZE and all of them on WRITE_SIZE
    s = _run(tmp_path, [131072.0])
    assert s["fetch_scale"] == pytest.approx(2.0) and s["write_scale"] == pytest.approx(1.0)
    assert s["fetch_bytes"] == pytest.approx(2.0 * 1000.0 * 1024)
    assert s["write_bytes"] == pytest.approx(3000.0 * 1024)
    assert s["avg_duration_us"] == pytest.approx(100.0)


def test_calibration_with_other_copies_on_the_grid_is_refused(tmp_path):
    with pytest.raises(ValueError, match="calibration copy"):
        _run(tmp_path, [131072.0, 4108.0])
