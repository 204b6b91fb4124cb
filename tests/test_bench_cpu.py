"""bench.py's contract checks that need no GPU: it refuses more than one GPU
with a message (the library has no multi-GPU path), and the stored traffic
record is complete (bench.py reports it only while the LBM kernel source
still has the recorded hash)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_complete():
    with open(os.path.join(ROOT, "profiles", "lbm_step_traffic.json")) as f:
        rec = json.load(f)
    assert rec["calibration"]["fetch_scale"] > 0 and rec["calibration"]["write_scale"] > 0
    for wl in ("c2", "c3"):
        r = rec[wl]
        assert len(r["source_hash"]) == 16 and r["dispatches"] > 0
        assert r["algorithmic_bytes_per_launch"] == 164 * r["fluid_nodes"]
        scaled = (r["fetch_kib_avg"] * rec["calibration"]["fetch_scale"] +
                  r["write_kib_avg"] * rec["calibration"]["write_scale"]) * 1024
        assert abs(scaled - r["hbm_bytes_per_launch"]) <= 1
        # HBM bytes within 1 % of the algorithmic 164 B per fluid node
        assert abs(r["ratio_to_algorithmic"] - 1.0) < 0.01
