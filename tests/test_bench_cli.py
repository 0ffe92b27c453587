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


def _tiled_layout_bytes(x):
    """sat2d's TILED layout of x (as include/cfar2d.h describes it), built on
    the host from its definition: FP32 sums inside 32 x 32 tiles, FP64 row
    lines S(32 I - 1, j) and column lines S(i, 32 J - 1)."""
    import numpy as np
    R, F = x.shape
    S = np.cumsum(np.cumsum(x, 0), 1)
    up = lambda v: (v + 255) // 256 * 256  # noqa: E731
    n_i, n_j = (R + 31) // 32, (F + 31) // 32
    loc = np.zeros((R, F))
    for i in range(R):
        for j in range(F):
            loc[i, j] = x[i // 32 * 32:i + 1, j // 32 * 32:j + 1].sum()
    rowl = np.zeros((n_i, F))
    coll = np.zeros((n_j, R))
    for i in range(1, n_i):
        rowl[i] = S[32 * i - 1]
    for j in range(1, n_j):
        coll[j] = S[:, 32 * j - 1]
    buf = np.zeros(up(R * F * 4) + up(n_i * F * 8) + up(n_j * R * 8), np.uint8)
    buf[:R * F * 4] = loc.astype(np.float32).view(np.uint8).ravel()
    o = up(R * F * 4)
    buf[o:o + n_i * F * 8] = rowl.view(np.uint8).ravel()
    o2 = o + up(n_i * F * 8)
    buf[o2:o2 + n_j * R * 8] = coll.view(np.uint8).ravel()
    return buf, o


def test_fp32_local_precision_measure():
    """The precision report's measure of the FP32-local integral image: zero
    on an integer map (every local sum exact), and it sees a corrupted carry."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    import oracle
    rng = np.random.default_rng(5)
    x = rng.integers(1, 50, size=(70, 90)).astype(np.float64)
    win = (2, 3, 5, 7, 1e-3)
    st = oracle.cfar2d(x, *win)[1]
    buf, row_off = _tiled_layout_bytes(x)
    assert bench.fp32_local_box_err(buf, 70, 90, win, st, block=16) == 0.0
    bad = buf.copy()
    lines = bad[row_off:row_off + 3 * 90 * 8].view(np.float64)
    lines[90 + 40] += 1.0  # S(31, 40) off by one
    assert bench.fp32_local_box_err(bad, 70, 90, win, st, block=16) > 1e-6
