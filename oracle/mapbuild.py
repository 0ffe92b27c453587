"""FP64 CPU oracle of the primary signal processing that makes the CA-CFAR
map from a raw radar record (Sec. II.A).

TEST INFRASTRUCTURE ONLY: the test suite may import this module; the product
path (``paper_2012_11077_amd``) never does, and the two share no code.

The record X has M fast-time samples (range) and N slow-time traces; it is
stored trace by trace: ``raw[n, m]``, n < N, m < M.  Steps, in the paper's
order, each a plain numpy definition:

1. fast time, per trace: DC-shift removal (subtract the trace mean), then
   linear-trend subtraction (least-squares line over m = 0..M-1);
2. slow time, per range bin: mean filter (centred moving average of odd
   length L, averaging only the samples inside the record at its ends), then
   normalisation (division by the largest magnitude of the filtered record,
   one scalar for the whole record; an all-zero record stays zero);
3. slow time, per range bin: discrete Fourier transform (numpy's FFT), power
   |F(k)|^2 (a square-law map, which eq. 2's CA-CFAR assumes), and the bins
   whose frequency k fs / N lies in [f_lo, f_hi] (0.3-0.8 Hz in the paper),
   k = ceil(f_lo N / fs) .. floor(f_hi N / fs).

The output map has M rows (range bins) and one column per kept bin.

Readings (the paper states the steps, not their parameters): L, the
normalisation's reference (global maximum magnitude) and the slow-time rate
fs are parameters; the band limits are inclusive; no window is applied before
the transform.
"""
from __future__ import annotations

import math

import numpy as np


def band_bins(n_traces: int, fs: float, f_lo: float, f_hi: float):
    """(k0, k1): the first and last DFT bin inside [f_lo, f_hi] (k1 < k0 if none)."""
    k0 = int(math.ceil(f_lo * n_traces / fs - 1e-9))
    k1 = int(math.floor(f_hi * n_traces / fs + 1e-9))
    k1 = min(k1, n_traces // 2)
    return k0, k1


def dc_detrend(raw: np.ndarray) -> np.ndarray:
    """Step 1: per trace (row of raw), subtract the mean, then the
    least-squares line over the sample index."""
    y = np.asarray(raw, dtype=np.float64)
    y = y - y.mean(axis=1, keepdims=True)
    M = y.shape[1]
    t = np.arange(M, dtype=np.float64)
    tc = t - t.mean()
    stt = float((tc * tc).sum())
    b = (y * tc).sum(axis=1, keepdims=True) / stt if stt > 0 else np.zeros((y.shape[0], 1))
    a = y.mean(axis=1, keepdims=True)
    return y - (a + b * tc)


def mean_filter(d: np.ndarray, L: int) -> np.ndarray:
    """Step 2a: d is range x slow time; centred moving average of odd length
    L along slow time, over the samples inside the record."""
    assert L >= 1 and L % 2 == 1
    h = L // 2
    R, N = d.shape
    out = np.empty_like(d)
    for n in range(N):
        lo, hi = max(0, n - h), min(N - 1, n + h)
        out[:, n] = d[:, lo:hi + 1].sum(axis=1) / (hi - lo + 1)
    return out


def build_map(raw: np.ndarray, fs: float, f_lo: float, f_hi: float, mean_len: int) -> np.ndarray:
    """Steps 1-3: the M x (k1 - k0 + 1) power map, float64."""
    N, M = raw.shape
    d = dc_detrend(raw).T                   # range x slow time
    g = mean_filter(d, mean_len)
    gmax = float(np.abs(g).max()) if g.size else 0.0
    if gmax > 0:
        g = g / gmax
    F = np.fft.fft(g, axis=1)
    k0, k1 = band_bins(N, fs, f_lo, f_hi)
    P = (F.real ** 2 + F.imag ** 2)[:, k0:k1 + 1]
    return np.ascontiguousarray(P)
