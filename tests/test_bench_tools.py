"""Host-side helpers of bench.py (CPU): the kernel-overlap summary of a
rocprofv3 kernel trace, on a synthetic trace whose busy and overlapping
times are known."""

import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Queue_Id", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_kernel_overlap_of_a_synthetic_trace(tmp_path):
    d = tmp_path / "trace" / "host"
    d.mkdir(parents=True)
    ms = 1_000_000
    rows = [
        # queue 1: [0, 10) and [20, 30) ms; queue 2: [5, 25) ms; a copy kernel is ignored
        {"Kernel_Name": "void hfx::k_eri<Eri1000, false, false, false>(hfx::QuartetArgs)", "Queue_Id": "1",
         "Start_Timestamp": 0, "End_Timestamp": 10 * ms},
        {"Kernel_Name": "void hfx::k_eri<Eri2221, false, false, false>(hfx::QuartetArgs)", "Queue_Id": "1",
         "Start_Timestamp": 20 * ms, "End_Timestamp": 30 * ms},
        {"Kernel_Name": "void hfx::k_eri<Eri1010, false, false, false>(hfx::QuartetArgs)", "Queue_Id": "2",
         "Start_Timestamp": 5 * ms, "End_Timestamp": 25 * ms},
        {"Kernel_Name": "__amd_rocclr_copyBuffer", "Queue_Id": "3", "Start_Timestamp": 0, "End_Timestamp": 40 * ms},
    ]
    _trace(d / "srv_kernel_trace.csv", rows)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--kernel-overlap", str(tmp_path / "trace")],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["dispatches"] == 3 and out["queues"] == 2
    assert abs(out["busy_ms"] - 30.0) < 1e-9      # union of [0,10), [5,25), [20,30)
    assert abs(out["overlap_ms"] - 10.0) < 1e-9   # [5,10) and [20,25)
    assert abs(out["overlap_fraction"] - 1.0 / 3.0) < 1e-12
