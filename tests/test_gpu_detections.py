"""Detection lists (cfar_detections) and bit-packed masks (cfar_mask_pack)
on the GPU, through the C ABI: record for record and bit for bit against the
oracle's definitions on the masks the detector wrote, capacity truncation,
empty masks, and properties at full size."""
import numpy as np
import pytest
import torch

import oracle
from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _detect(spec):
    x = torch.from_numpy(synth.generate(spec)).to(DEV)
    mask = torch.empty(x.shape, dtype=torch.uint8, device=DEV)
    thr = torch.empty(x.shape, dtype=torch.float64, device=DEV)
    C.cfar2d(x, spec.window, C.TILED, mask=mask, threshold=thr)
    return x, mask, thr


def _records(d):
    return list(zip(d["row"].cpu().tolist(), d["col"].cpu().tolist(), d["cut"].cpu().tolist(),
                    d["threshold"].cpu().tolist()))


def _same(got, want):
    assert len(got) == len(want)
    for g, w in zip(got, want):
        assert g[:3] == w[:3], (g, w)
        assert (np.isnan(g[3]) and np.isnan(w[3])) or g[3] == w[3], (g, w)


@pytest.mark.parametrize("shape", [(1, 1), (37, 29), (300, 5000), (64, 4096), (5, 8193)])
def test_list_matches_oracle(shape):
    R, F = shape
    spec = synth.MapSpec(R, F, "f32", "exp", 1.0, n_targets=8, guard_r=1, guard_f=1, train_r=3, train_f=3,
                         pfa=1e-2, seed=(81, R, F))
    x, mask, thr = _detect(spec)
    d = C.detections(x, mask, threshold=thr)
    torch.cuda.synchronize()
    m_np, x_np, t_np = mask.cpu().numpy(), x.cpu().numpy().astype(np.float64), thr.cpu().numpy()
    want = oracle.detection_list(m_np, x_np, t_np)
    say("detections", shape, d["count"])
    assert d["count"] == int(m_np.sum()) == len(want)
    _same(_records(d), want)
    # without a threshold output the threshold field is NaN
    d2 = C.detections(x, mask)
    torch.cuda.synchronize()
    _same(_records(d2), [(r, c, v, float("nan")) for (r, c, v, _) in want])


def test_capacity_and_empty():
    spec = synth.MapSpec(200, 300, "f64", "exp", 1.0, n_targets=5, guard_r=1, guard_f=1, train_r=2, train_f=2,
                         pfa=1e-2, seed=(82,))
    x, mask, thr = _detect(spec)
    full = C.detections(x, mask, threshold=thr)
    n = full["count"]
    assert n > 10
    half = C.detections(x, mask, threshold=thr, capacity=n // 2)
    none = C.detections(x, mask, capacity=0)
    torch.cuda.synchronize()
    assert half["count"] == n and none["count"] == n
    _same(_records(half), _records(full)[: n // 2])
    zero = torch.zeros_like(mask)
    e = C.detections(x, zero)
    torch.cuda.synchronize()
    assert e["count"] == 0 and len(e["row"]) == 0


@pytest.mark.parametrize("cols", [1, 31, 32, 33, 1000])
def test_pack_matches_oracle(cols):
    spec = synth.MapSpec(50, cols, "f32", "exp", 1.0, n_targets=3, guard_r=1, guard_f=0, train_r=2, train_f=1,
                         pfa=0.05, seed=(83, cols))
    x, mask, _ = _detect(spec)
    bits = C.mask_pack(x, mask)
    torch.cuda.synchronize()
    want = oracle.pack_mask(mask.cpu().numpy())
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), want)


def test_pack_strided_mask():
    """A mask view with ld_mask > cols: only its own columns are packed."""
    x = torch.rand((40, 70), dtype=torch.float32, device=DEV)
    big = torch.zeros((40, 100), dtype=torch.uint8, device=DEV)
    big[:, 70:] = 1                    # outside the view
    mv = big[:, :70]
    mv.copy_((torch.rand((40, 70), device=DEV) < 0.3).to(torch.uint8))
    bits = C.mask_pack(x, mv)
    torch.cuda.synchronize()
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), oracle.pack_mask(mv.cpu().numpy()))


def test_full_size_properties():
    """16384 x 16384 FP32 at Pfa 1e-3: the count equals the mask's sum, the
    records are strictly increasing in row-major order and each is a set
    cell with its own CUT; the packed mask unpacks to the mask."""
    spec = synth.MapSpec(16384, 16384, "f32", "exp", 2.0, n_targets=500, guard_r=2, guard_f=2, train_r=8,
                         train_f=8, pfa=1e-3, seed=(84,))
    x, mask, thr = _detect(spec)
    say("full-size detections")
    d = C.detections(x, mask, threshold=thr)
    torch.cuda.synchronize()
    total = int(mask.sum().item())
    assert d["count"] == total and total > 100000
    key = d["row"].to(torch.int64) * 16384 + d["col"].to(torch.int64)
    assert bool((key[1:] > key[:-1]).all().item())
    rows, cols = d["row"].to(torch.int64), d["col"].to(torch.int64)
    assert bool((mask[rows, cols] == 1).all().item())
    assert bool((x[rows, cols].double() == d["cut"]).all().item())
    assert bool((thr[rows, cols] == d["threshold"]).all().item())
    bits = C.mask_pack(x, mask)
    sh = torch.arange(32, device=DEV, dtype=torch.int32)
    unpacked = ((bits.unsqueeze(-1) >> sh) & 1).reshape(16384, -1)[:, :16384].to(torch.uint8)
    torch.cuda.synchronize()
    assert torch.equal(unpacked, mask)
