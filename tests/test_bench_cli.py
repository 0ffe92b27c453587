"""bench.py's command line without a GPU: more than one GPU is refused with a
message, and the traffic files parse and name the kernel source they were
measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_files_are_well_formed():
    for name in ("fused_kernel_uneven_batch_traffic.json", "fused_kernel_16k_f32_map_traffic.json",
                 "fused_kernel_8k_f64_map_traffic.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
        assert t["kernel"] == "fused_kernel" and len(t["kernel_sha"]) == 16
        assert t["bytes_per_launch"] > 0 and t["fetch_scale"] > 0 and t["write_scale"] > 0
