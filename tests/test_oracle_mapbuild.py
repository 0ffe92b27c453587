"""Pins of the map-building oracle (Sec. II.A: DC removal, linear detrend,
mean filter, normalisation, DFT, power, respiration band): brute force on
tiny records with loops written independently of the oracle, a library
detrend, closed forms for tones and lines, scale invariance, and the
breathing target of a synthetic record showing up at its range and rate."""
import cmath
import math

import numpy as np
import pytest
from scipy.signal import detrend as scipy_detrend

from oracle import mapbuild as MB
from paper_2012_11077_amd import synth


def _brute(raw, fs, f_lo, f_hi, L):
    N, M = raw.shape
    d = [[0.0] * N for _ in range(M)]
    tm = (M - 1) / 2.0
    stt = sum((t - tm) ** 2 for t in range(M))
    for n in range(N):
        mean = sum(float(raw[n, t]) for t in range(M)) / M
        y = [float(raw[n, t]) - mean for t in range(M)]
        b = sum((t - tm) * y[t] for t in range(M)) / stt if stt > 0 else 0.0
        ym = sum(y) / M
        for t in range(M):
            d[t][n] = y[t] - (ym + b * (t - tm))
    h = L // 2
    g = [[0.0] * N for _ in range(M)]
    for m in range(M):
        for n in range(N):
            idx = [j for j in range(n - h, n + h + 1) if 0 <= j < N]
            g[m][n] = sum(d[m][j] for j in idx) / len(idx)
    gmax = max(abs(v) for row in g for v in row) or 1.0   # an all-zero record stays zero
    k0 = math.ceil(f_lo * N / fs - 1e-9)
    k1 = min(math.floor(f_hi * N / fs + 1e-9), N // 2)
    out = np.zeros((M, max(0, k1 - k0 + 1)))
    for m in range(M):
        for k in range(k0, k1 + 1):
            s = sum((g[m][n] / gmax) * cmath.exp(-2j * math.pi * k * n / N) for n in range(N))
            out[m, k - k0] = abs(s) ** 2
    return out


@pytest.mark.parametrize("N, M, L", [(12, 5, 3), (16, 7, 1), (9, 4, 5), (20, 1, 3)])
def test_brute_force_tiny(N, M, L):
    rng = np.random.default_rng(N * 100 + M)
    raw = rng.standard_normal((N, M)) + 0.3 * np.arange(M)[None, :]
    fs, f_lo, f_hi = 4.0, 0.3, 1.7
    want = _brute(raw, fs, f_lo, f_hi, L)
    got = MB.build_map(raw, fs, f_lo, f_hi, L)
    assert got.shape == want.shape
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12 * max(1.0, want.max()))


def test_detrend_matches_library_and_removes_lines():
    rng = np.random.default_rng(1)
    raw = rng.standard_normal((7, 33))
    np.testing.assert_allclose(MB.dc_detrend(raw), scipy_detrend(raw, axis=1, type="linear"), atol=1e-12)
    lines = 2.0 + 0.5 * np.arange(33)[None, :] * rng.standard_normal((7, 1))
    assert np.abs(MB.dc_detrend(lines)).max() < 1e-12


def test_mean_filter_closed_forms():
    d = np.full((3, 10), 2.5)
    np.testing.assert_allclose(MB.mean_filter(d, 5), d)
    x = np.arange(10, dtype=np.float64)[None, :]
    np.testing.assert_array_equal(MB.mean_filter(x, 1), x)
    f = MB.mean_filter(x, 3)
    assert f[0, 0] == 0.5 and f[0, 5] == 5.0 and f[0, 9] == 8.5   # ends average 2 samples


def test_tone_power_closed_form():
    """A slow-time cosine at bin k in every range bin of an otherwise
    constant-in-fast-time record: after normalisation (peak 1) the power at
    bin k is (N/2)^2 and the other kept bins are ~0."""
    N, M, k = 64, 8, 5
    n = np.arange(N)
    tone = np.cos(2 * np.pi * k * n / N)
    # vary with range so the detrend (per trace, over range) keeps it
    prof = np.cos(np.pi * np.arange(M) / 2.0)
    raw = tone[:, None] * prof[None, :]
    P = MB.build_map(raw, fs=float(N), f_lo=1.0, f_hi=10.0, mean_len=1)
    d = MB.dc_detrend(raw).T
    peak = np.abs(d).max()
    for m in range(M):
        amp = np.abs(d[m]).max() / peak
        assert P[m, k - 1] == pytest.approx((amp * N / 2) ** 2, rel=1e-9, abs=1e-9)
        assert np.delete(P[m], k - 1).max() < 1e-18 + 1e-12 * P[m, k - 1]


def test_band_bins_and_scale_invariance():
    assert MB.band_bins(600, 20.0, 0.3, 0.8) == (9, 24)
    assert MB.band_bins(600, 20.0, 0.31, 0.32)[1] < MB.band_bins(600, 20.0, 0.31, 0.32)[0]  # empty band
    rng = np.random.default_rng(2)
    raw = rng.standard_normal((40, 9))
    np.testing.assert_allclose(MB.build_map(7.5 * raw, 10.0, 0.5, 3.0, 3), MB.build_map(raw, 10.0, 0.5, 3.0, 3),
                               rtol=1e-12)
    assert not MB.build_map(np.zeros((40, 9)), 10.0, 0.5, 3.0, 3).any()


def test_breathing_target_is_at_its_range_and_rate():
    spec = synth.RawSpec(n_traces=600, n_samples=512, target_bin=300, seed=(3,))
    raw = synth.generate_raw(spec)
    P = MB.build_map(raw, spec.fs_slow, 0.3, 0.8, 5)
    k0, _ = MB.band_bins(600, spec.fs_slow, 0.3, 0.8)
    m, j = np.unravel_index(np.argmax(P), P.shape)
    assert abs(m - 300) <= spec.pulse_width and j + k0 == round(0.3 * 600 / spec.fs_slow)
