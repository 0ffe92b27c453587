"""Building the CA-CFAR map from a raw record on the GPU (cfar_map_build,
Sec. II.A) against the oracle's steps, through the C ABI: record shapes
and types, strided records, the all-zero record, and the whole chain on a
record of the paper's size (600 traces x 1024 samples) down to the
detection of the breathing target."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mapbuild as MB
from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import check_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _cmp(got, want, rel):
    scale = max(float(np.abs(want).max()), 1e-300)
    err = float(np.abs(got.astype(np.float64) - want).max()) / scale
    assert err <= rel, err
    return err


@pytest.mark.parametrize("N, M, L, fs, band", [
    (600, 1024, 5, 20.0, (0.3, 0.8)),     # the paper's record size
    (64, 33, 1, 8.0, (0.5, 3.0)),
    (101, 7, 9, 10.0, (0.0, 5.0)),        # odd N, DC and Nyquist bins
    (4000, 17, 31, 50.0, (0.3, 0.8)),     # the largest record length
    (3, 1, 3, 2.0, (0.0, 1.0)),           # one sample per trace: zero map
])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_matches_oracle(N, M, L, fs, band, dtype):
    rng = np.random.default_rng(N + M)
    raw = (rng.standard_normal((N, M)) + 0.01 * np.arange(M)[None, :]).astype(np.float32 if dtype == "f32" else np.float64)
    want = MB.build_map(raw, fs, band[0], band[1], L)
    x = torch.from_numpy(raw).to(DEV)
    for out_dtype, rel in ((torch.float64, 1e-10), (torch.float32, 1e-6)):
        got = C.build_map(x, fs, band[0], band[1], L, out_dtype=out_dtype)
        torch.cuda.synchronize()
        say("mapbuild", N, M, L, dtype, out_dtype, tuple(got.shape))
        assert tuple(got.shape) == want.shape
        _cmp(got.cpu().numpy(), want, rel)


def test_strided_and_zero_records():
    rng = np.random.default_rng(5)
    big = torch.from_numpy(rng.standard_normal((200, 90)).astype(np.float32)).to(DEV)
    view = big[:, 5:75]                                   # ld_raw = 90 > 70 samples
    want = MB.build_map(view.cpu().numpy(), 10.0, 0.2, 2.0, 3)
    got = C.build_map(view, 10.0, 0.2, 2.0, 3, out_dtype=torch.float64)
    torch.cuda.synchronize()
    _cmp(got.cpu().numpy(), want, 1e-10)
    z = C.build_map(torch.zeros((50, 40), device=DEV), 10.0, 0.2, 2.0, 3)
    torch.cuda.synchronize()
    assert not bool(z.any().item())


def test_paper_record_to_detection():
    """600 x 1024 record with a breathing target at range sample 700:
    GPU map = oracle map; CA-CFAR on it (TILED, guard 2, training 4 per
    side, Pfa 1e-4) equals the oracle's decisions outside the margin and
    detects the target at 0.3 Hz."""
    spec = synth.RawSpec(n_traces=600, n_samples=1024, target_bin=700, seed=(11,))
    raw = synth.generate_raw(spec)
    want = MB.build_map(raw, spec.fs_slow, 0.3, 0.8, 5)
    x = torch.from_numpy(raw).to(DEV)
    m = C.build_map(x, spec.fs_slow, 0.3, 0.8, 5, out_dtype=torch.float64)
    torch.cuda.synchronize()
    m_np = m.cpu().numpy()
    _cmp(m_np, want, 1e-10)
    win = (2, 2, 4, 4, 1e-4)
    mask = C.cfar2d(m, win, C.TILED)
    torch.cuda.synchronize()
    mk = mask.cpu().numpy()
    check_full(m_np, win, mk)
    ref = oracle.cfar2d(want, *win)[0]
    k0, _ = C.map_bins(600, spec.fs_slow)
    jb = round(0.3 * 600 / spec.fs_slow) - k0
    rows = np.nonzero(mk[:, jb])[0]
    say("detections at 0.3 Hz:", rows.tolist()[:20], "oracle:", np.nonzero(ref[:, jb])[0].tolist()[:20])
    assert np.any(np.abs(rows - 700) <= spec.pulse_width)
