"""Host checks of the rocprofv3 CSV summariser (no GPU needed): kernel statistics from
a trace, counter means, and the per-grid split that separates the launches doing work
from the empty ones at the end of a batched solve."""
import csv
import os

from paper_1903_08741_amd import prof_summary as ps

TRACE_COLS = ["Kind", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y"]
PMC_COLS = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]


def _write(path, cols, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))


def test_trace_tables(tmp_path):
    d = tmp_path / "run"
    d.mkdir()
    k = "void rmg::k_down<float, 32, 2>(rmg::SolveArgs, rmg::StreamPlan)"
    rows = [("KERNEL", k, 0, 10000, 65536, 64), ("KERNEL", k, 0, 12000, 65536, 64),
            ("KERNEL", k, 0, 1000, 65536, 64),  # an empty launch: below half the maximum
            ("KERNEL", k, 0, 3000, 16384, 64), ("KERNEL", "void other()", 0, 4000, 256, 1)]
    _write(os.path.join(d, "run_kernel_trace.csv"), TRACE_COLS, rows)
    flat = ps.kernel_table(str(tmp_path), "")
    assert flat[2].startswith("| k_down<float, 32, 2> | 4 | 0.0 | 6.50 |"), flat
    by = ps.grid_kernel_table(str(tmp_path), "k_down")
    assert "| k_down<float, 32, 2> | 65536x64 | 3 | 7.67 | 2 | 11.00 |" in by, by
    assert "| k_down<float, 32, 2> | 16384x64 | 1 | 3.00 | 1 | 3.00 |" in by, by
    assert not any("other" in line for line in by)


def test_counter_tables(tmp_path):
    d = tmp_path / "pmc"
    d.mkdir()
    k = "rmg::k_up<float, 32, 2>(rmg::SolveArgs)"
    rows = [(k, 4194304, "FETCH_SIZE", 100.0), (k, 4194304, "FETCH_SIZE", 300.0),
            (k, 4194304, "FETCH_SIZE", 20.0), (k, 262144, "FETCH_SIZE", 7.0)]
    _write(os.path.join(d, "run_counter_collection.csv"), PMC_COLS, rows)
    flat = ps.counter_table(str(tmp_path), "")
    assert "| k_up<float, 32, 2> | FETCH_SIZE | 4 | 106.75 | 427 |" in flat, flat
    by = ps.grid_counter_table(str(tmp_path), "")
    assert "| k_up<float, 32, 2> | 4194304 | FETCH_SIZE | 3 | 140 | 1 | 300 |" in by, by
    assert "| k_up<float, 32, 2> | 262144 | FETCH_SIZE | 1 | 7 | 1 | 7 |" in by, by
