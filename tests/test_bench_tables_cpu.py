"""Host logic of bench.py's kernel table (no GPU): launches of a rocprofv3
kernel trace are assigned to the fixed-grid layouts by the step launches,
which run under either name of the step kernel."""
import csv
import io
import json
import os
import sys
from contextlib import redirect_stdout

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _trace(path, step_name, phases, per):
    """A trace of `per` evaluations per layout: k_gather then the step, 10 us
    apart; the gather's duration encodes the layout (100 + layout index us)."""
    t = 1_000_000  # rocprofv3 timestamps are positive
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for p in range(len(phases)):
            for _ in range(per):
                for name, dur in (("tsnet::k_gather(int)", (100 + p) * 1000),
                                  (f"tsnet::{step_name}(int)", 5000)):
                    w.writerow({"Kernel_Name": name, "Start_Timestamp": t, "End_Timestamp": t + dur})
                    t += 10_000_000


@pytest.mark.parametrize("step_name", ["k_step", "k_step_pairs"])
def test_kernel_table_splits_layouts_by_step(tmp_path, step_name):
    per = bench.FIXED_GRID_EVALS
    phases = [{"std": 6.0, "n_int": 256, "evals": per}, {"std": 12.0, "n_int": 512, "evals": per}]
    _trace(tmp_path / "trace.csv", step_name, phases, per)
    info = tmp_path / "info.json"
    info.write_text(json.dumps({"n": 1000, "nnz": 5000, "phases": phases}))
    out = io.StringIO()
    with redirect_stdout(out):
        bench.kernel_table(str(tmp_path / "trace.csv"), str(info))
    rows = [r for r in out.getvalue().splitlines() if r.startswith("| k_")]
    gather = {r.split("|")[2].strip(): float(r.split("|")[4]) for r in rows if r.startswith("| k_gather")}
    assert gather == {"256": 100.0, "512": 101.0}
    steps = [r for r in rows if r.startswith(f"| {step_name} ")]
    assert len(steps) == 2 and all("| 56,000 |" in r for r in steps)
