"""bench.py's contract, checked on the CPU: the one-GPU refusal, the work
model's bytes, and the lookup of the dominant kernel's committed HBM
traffic under the name the kernel runs as on the current sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout.strip()


def test_work_model_bytes():
    # 4 B per wedge check, 4 B per hit (metadata), 9 B (4 B) per staged
    # out-list entry, 8 B per in-edge record, 16 B per tile
    st = {"class_probes": [10, 20, 30, 40], "class_staged": [1, 2, 3, 4], "class_records": [5, 6, 7, 8],
          "class_tiles": [9, 10, 11, 12]}
    assert bench.algorithmic_bytes(st, 2, True, 100) == 4 * 30 + 4 * 100 + 9 * 3 + 8 * 7 + 16 * 11
    assert bench.algorithmic_bytes(st, 2, False, 100) == 4 * 30 + 4 * 3 + 8 * 7 + 16 * 11


def test_dominant_kernel_traffic_is_current():
    # the scale-26 workload's large class: the kernel name the line reports is
    # one the committed counter summary measured, on these very sources
    rec = json.load(open(bench.TRAFFIC_FILE))
    key = bench.kernel_key(2, 0, True)
    assert key in rec["kernels"], (key, sorted(rec["kernels"]))
    assert rec["kernel_hash"] == bench.kernel_source_hash()
    assert bench.load_traffic(key, rec["workload"]) == int(rec["kernels"][key]["hbm_bytes_per_launch"])
