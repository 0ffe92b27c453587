"""Seeded synthetic range x slow-time-frequency power maps.

This module only draws inputs.  It holds none of the detector's arithmetic
(no integral image, no window sums, no thresholds), so the FP64 oracle and the
HIP path can both be fed from it without sharing any of the method.

The paper's own records (600 traces x 1024 samples of UWB radar, Sec. III)
are not available, so every map here is synthetic: a square-law (power) map
of the band-limited slow-time spectrum per range bin (Sec. II.A), i.e. rows =
range bins, columns = frequency bins, frequency contiguous in memory.

Clutter models
  * ``exp``       i.i.d. exponential power with a constant mean (the noise law
                  under which CA-CFAR holds its false-alarm rate);
  * ``exp_ramp``  exponential with mean 10**(2 i / (R-1)), i.e. 0 dB to 20 dB
                  across range, flat in frequency;
  * ``lognormal`` exp(sigma * N(0,1)), sigma in natural-log units (sigma = 2
                  spans about 60 dB), mean exp(sigma**2 / 2).
Targets: a 3 x 3 footprint centred on a uniformly drawn cell, weights
[0.5, 1, 0.5] x [0.5, 1, 0.5] (centre 1), amplitude = local clutter mean x
10**(SNR/10), clipped at the border.  Draw order per map: clutter, target
cells, target SNRs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

DTYPES = {"f32": np.float32, "f64": np.float64}


@dataclasses.dataclass(frozen=True)
class MapSpec:
    """One synthetic map and the CFAR window it is run with."""

    rows: int
    cols: int
    dtype: str = "f32"             # "f32" or "f64": the storage type of the map
    clutter: str = "exp"           # "exp" | "exp_ramp" | "lognormal"
    mean: float = 1.0              # exp: clutter mean power
    sigma: float = 2.0             # lognormal: sigma in natural-log units
    n_targets: int = 0
    snr_lo_db: float = 10.0
    snr_hi_db: float = 25.0
    guard_r: int = 2
    guard_f: int = 2
    train_r: int = 8
    train_f: int = 8
    pfa: float = 1e-4
    seed: Sequence[int] = (0,)

    @property
    def cells(self) -> int:
        return self.rows * self.cols

    @property
    def window(self):
        return (self.guard_r, self.guard_f, self.train_r, self.train_f, self.pfa)


def _rng(seed) -> np.random.Generator:
    return np.random.default_rng(list(seed) if isinstance(seed, (tuple, list)) else seed)


def _clutter_mean(spec: MapSpec, i: np.ndarray) -> np.ndarray:
    """Local clutter mean power at range bins ``i`` (used to scale targets)."""
    if spec.clutter == "exp":
        return np.full(i.shape, spec.mean, dtype=np.float64)
    if spec.clutter == "exp_ramp":
        if spec.rows == 1:
            return np.ones(i.shape, dtype=np.float64)
        return 10.0 ** (2.0 * i / (spec.rows - 1))
    if spec.clutter == "lognormal":
        return np.full(i.shape, math.exp(spec.sigma ** 2 / 2.0), dtype=np.float64)
    raise ValueError("unknown clutter model %r" % spec.clutter)


def generate(spec: MapSpec, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Draw the map described by ``spec`` (C-contiguous, rows x cols, spec.dtype)."""
    return generate_with_targets(spec, out)[0]


def generate_with_targets(spec: MapSpec, out: Optional[np.ndarray] = None):
    """Draw the map and return ``(map, targets)``, targets an (n, 3) array of
    (row, col, snr_db) of the planted point targets."""
    dt = DTYPES[spec.dtype]
    rng = _rng(spec.seed)
    R, F = spec.rows, spec.cols
    if out is None:
        out = np.empty((R, F), dtype=dt)
    assert out.shape == (R, F) and out.dtype == dt
    if spec.clutter in ("exp", "exp_ramp"):
        rng.standard_exponential(size=(R, F), dtype=dt, out=out)
        if spec.clutter == "exp":
            if spec.mean != 1.0:
                out *= dt(spec.mean)
        else:
            out *= _clutter_mean(spec, np.arange(R, dtype=np.float64)).astype(dt)[:, None]
    elif spec.clutter == "lognormal":
        rng.standard_normal(size=(R, F), dtype=dt, out=out)
        out *= dt(spec.sigma)
        np.exp(out, out=out)
    else:
        raise ValueError("unknown clutter model %r" % spec.clutter)
    n = spec.n_targets
    targets = np.zeros((0, 3))
    if n > 0:
        ti = rng.integers(0, R, size=n)
        tj = rng.integers(0, F, size=n)
        snr = rng.uniform(spec.snr_lo_db, spec.snr_hi_db, size=n)
        amp = _clutter_mean(spec, ti.astype(np.float64)) * 10.0 ** (snr / 10.0)
        w = (0.5, 1.0, 0.5)
        for k in range(n):
            for di in (-1, 0, 1):
                a = ti[k] + di
                if a < 0 or a >= R:
                    continue
                for dj in (-1, 0, 1):
                    b = tj[k] + dj
                    if b < 0 or b >= F:
                        continue
                    out[a, b] += dt(amp[k] * w[di + 1] * w[dj + 1])
        targets = np.stack([ti.astype(np.float64), tj.astype(np.float64), snr], axis=1)
    return out, targets


# ---------------------------------------------------------------------------
# The benchmark workloads.  Sizes and distributions follow the stated configs;
# seeds are the config index.
# ---------------------------------------------------------------------------

def config0() -> MapSpec:
    """One 512 x 256 FP64 map, Exp(1) clutter, 5 targets at 15 dB, guard 2x2,
    training 8x8, Pfa 1e-4, seed 0."""
    return MapSpec(512, 256, "f64", "exp", 1.0, n_targets=5, snr_lo_db=15.0, snr_hi_db=15.0,
                   guard_r=2, guard_f=2, train_r=8, train_f=8, pfa=1e-4, seed=(0,))


def config1(rows: int = 8192, cols: int = 8192) -> MapSpec:
    """8192 x 8192 FP64, exponential clutter on a 0-20 dB range ramp, 200
    targets at 10-25 dB, guard 3x3, training 16x16, Pfa 1e-6, seed 1."""
    nt = max(1, round(200 * rows * cols / (8192 * 8192)))
    return MapSpec(rows, cols, "f64", "exp_ramp", n_targets=nt, snr_lo_db=10.0, snr_hi_db=25.0,
                   guard_r=3, guard_f=3, train_r=16, train_f=16, pfa=1e-6, seed=(1,))


def config2(rows: int = 16384, cols: int = 16384) -> MapSpec:
    """16384 x 16384 FP32, log-normal clutter (sigma 2), 1000 targets at
    8-30 dB, guard 4x4, training 24x24, Pfa 1e-5, seed 2."""
    nt = max(1, round(1000 * rows * cols / (16384 * 16384)))
    return MapSpec(rows, cols, "f32", "lognormal", sigma=2.0, n_targets=nt, snr_lo_db=8.0,
                   snr_hi_db=30.0, guard_r=4, guard_f=4, train_r=24, train_f=24, pfa=1e-5,
                   seed=(2,))


def config3_specs(n: int = 512, seed: int = 3, rows=(200, 4096), cols=(64, 2048),
                  dtype: str = "f32") -> List[MapSpec]:
    """The uneven batch: ``n`` maps with rows ~ U[200, 4096], cols ~ U[64, 2048],
    exponential clutter with mean log-uniform in [0.1, 10], 0-20 targets at
    10-25 dB, per-axis guard in 1..4 and training in 4..24, Pfa in
    {1e-3, 1e-4, 1e-6}.  Map k is drawn from seed (seed, k + 1), so any map
    can be regenerated on its own."""
    rng = _rng((seed,))
    R = rng.integers(rows[0], rows[1] + 1, size=n)
    F = rng.integers(cols[0], cols[1] + 1, size=n)
    mean = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=n))
    ntg = rng.integers(0, 21, size=n)
    gr = rng.integers(1, 5, size=n)
    gf = rng.integers(1, 5, size=n)
    tr = rng.integers(4, 25, size=n)
    tf = rng.integers(4, 25, size=n)
    pfa = rng.choice(np.array([1e-3, 1e-4, 1e-6]), size=n)
    return [MapSpec(int(R[k]), int(F[k]), dtype, "exp", float(mean[k]), n_targets=int(ntg[k]),
                    snr_lo_db=10.0, snr_hi_db=25.0, guard_r=int(gr[k]), guard_f=int(gf[k]),
                    train_r=int(tr[k]), train_f=int(tf[k]), pfa=float(pfa[k]),
                    seed=(seed, k + 1))
            for k in range(n)]


def config4_streams(n_streams: int = 16, seed: int = 4) -> List[dict]:
    """The serving workload: ``n_streams`` drone streams, stream k emitting
    frames of (round(256 * 2**(4k/15)), round(128 * 2**(3k/15))) FP32 cells
    (256 x 128 up to 4096 x 1024) at Poisson rate 50 Hz; clutter, targets,
    window and Pfa of each frame drawn as for the uneven batch."""
    out = []
    last = max(1, n_streams - 1)
    for k in range(n_streams):
        R = int(round(256 * 2.0 ** (4.0 * k / last)))
        F = int(round(128 * 2.0 ** (3.0 * k / last)))
        out.append({"stream": k, "rows": R, "cols": F, "rate_hz": 50.0, "seed": seed})
    return out


def stream_frame_spec(stream: dict, frame: int) -> MapSpec:
    """Frame ``frame`` of a serving stream, drawn from seed
    (seed, stream, frame) with the uneven batch's distributions: exponential
    clutter with mean log-uniform in [0.1, 10], 0-20 targets at 10-25 dB,
    per-axis guard in 1..4 and training in 4..24, Pfa in {1e-3, 1e-4, 1e-6}."""
    R, F = stream["rows"], stream["cols"]
    rng = _rng((stream["seed"], stream["stream"], frame, 7))
    mean = float(np.exp(rng.uniform(math.log(0.1), math.log(10.0))))
    gr, gf = (int(v) for v in rng.integers(1, 5, size=2))
    tr, tf = (int(v) for v in rng.integers(4, 25, size=2))
    pfa = float(rng.choice(np.array([1e-3, 1e-4, 1e-6])))
    return MapSpec(R, F, "f32", "exp", mean, n_targets=int(rng.integers(0, 21)), snr_lo_db=10.0,
                   snr_hi_db=25.0, guard_r=gr, guard_f=gf, train_r=tr, train_f=tf, pfa=pfa,
                   seed=(stream["seed"], stream["stream"], frame))


def random_small_specs(n: int, seed: int, max_rows: int = 96, max_cols: int = 96,
                       dtype: str = "f32") -> List[MapSpec]:
    """Small maps of random shape and window (for parity tests), including
    windows wider than the map, zero guard or zero training on one axis."""
    rng = _rng((seed, 99))
    out = []
    for k in range(n):
        R = int(rng.integers(1, max_rows + 1))
        F = int(rng.integers(1, max_cols + 1))
        gr, gf = (int(v) for v in rng.integers(0, 5, size=2))
        tr, tf = (int(v) for v in rng.integers(0, 13, size=2))
        if tr + tf == 0:
            tf = 1
        pfa = float(rng.choice([1e-1, 1e-2, 1e-3, 1e-4, 1e-6]))
        out.append(MapSpec(R, F, dtype, "exp", float(np.exp(rng.uniform(-2, 2))),
                           n_targets=int(rng.integers(0, 4)), snr_lo_db=5.0, snr_hi_db=25.0,
                           guard_r=gr, guard_f=gf, train_r=tr, train_f=tf, pfa=pfa,
                           seed=(seed, k)))
    return out


# ---------------------------------------------------------------------------
# Raw radar records (the input of the primary signal processing, Sec. II.A):
# N traces of M fast-time samples, stored trace by trace.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class RawSpec:
    """One synthetic UWB record: static clutter, a per-trace DC offset and
    fast-time drift, white noise, and a breathing target whose echo (a
    Gaussian monocycle) moves back and forth in range at the breathing
    rate."""

    n_traces: int = 600            # slow time (the paper: 600 traces)
    n_samples: int = 1024          # fast time (the paper: 1024 samples)
    fs_slow: float = 20.0          # traces per second (not stated in the paper)
    target_bin: int = 400          # range sample of the target's echo
    target_amp: float = 1.0
    breath_hz: float = 0.3         # the paper's actuator: 0.3 Hz
    breath_samples: float = 1.3    # peak displacement in fast-time samples (~1 cm at 39 GS/s)
    pulse_width: float = 6.0       # monocycle width in samples
    clutter_amp: float = 3.0
    noise: float = 0.05
    dc_sigma: float = 0.2
    drift_sigma: float = 1e-3
    dtype: str = "f32"
    seed: Sequence[int] = (9,)


def generate_raw(spec: RawSpec) -> np.ndarray:
    """Draw the record, shape (n_traces, n_samples).  Draw order: clutter
    profile, DC offsets, drifts, breathing phase, noise."""
    rng = _rng(spec.seed)
    N, M = spec.n_traces, spec.n_samples
    m = np.arange(M, dtype=np.float64)
    clutter = spec.clutter_amp * rng.standard_normal(M) * np.exp(-m / max(1.0, M / 4.0))
    dc = spec.dc_sigma * rng.standard_normal(N)
    drift = spec.drift_sigma * rng.standard_normal(N)
    phase = rng.uniform(0.0, 2.0 * math.pi)
    noise = spec.noise * rng.standard_normal((N, M))
    t = np.arange(N, dtype=np.float64) / spec.fs_slow
    centre = spec.target_bin + spec.breath_samples * np.sin(2.0 * math.pi * spec.breath_hz * t + phase)
    u = (m[None, :] - centre[:, None]) / spec.pulse_width
    echo = spec.target_amp * (-u) * np.exp(-0.5 * u * u)          # Gaussian monocycle
    raw = clutter[None, :] + dc[:, None] + drift[:, None] * m[None, :] + echo + noise
    return raw.astype(DTYPES[spec.dtype])
