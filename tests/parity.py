"""Parity rule between the HIP path and the FP64 oracle.

* A cell is near-threshold when |X - T_oracle| <= 1e-5 |T_oracle|; both
  decisions are accepted there, and such cells are counted.
* Every other cell's mask must match the oracle bit for bit.
* Training sums: TILED and DIRECT forms within 1e-6 relative of the oracle
  (the bound the precision form is held to); PLAIN form within the rounding of an FP64
  integral image, 64 * eps64 * (sum of the map) plus 1e-12 relative, since
  both sides take differences of SAT entries that grow with the map.
"""
import sys

import numpy as np

import oracle

EPS64 = np.finfo(np.float64).eps
TILED_REL = 1e-6
MARGIN = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_full(x_np, window, mask, st=None, thr=None, form="tiled", ref=None):
    """Compare a whole map.  Returns dict(near=..., max_rel=...)."""
    gr, gf, tr, tf, pfa = window
    if ref is None:
        ref = oracle.cfar2d(x_np, gr, gf, tr, tf, pfa)
    m_o, st_o, nt_o, thr_o = ref
    near = oracle.near_threshold(x_np, thr_o, MARGIN)
    bad = (mask != m_o) & ~near
    assert not bad.any(), "mask mismatch outside margin at %s (of %d)" % (
        np.argwhere(bad)[:5].tolist(), int(bad.sum()))
    out = {"near": int(near.sum()), "max_rel": 0.0, "detections": int(m_o.sum())}
    if st is not None:
        err = np.abs(st - st_o)
        if form in ("tiled", "direct"):
            tol = TILED_REL * np.abs(st_o)
        else:
            tol = 64 * EPS64 * float(np.abs(np.asarray(x_np, dtype=np.float64)).sum()) + 1e-12 * np.abs(st_o)
        tol = np.maximum(tol, 1e-300)
        worst = np.argmax(err - tol)
        assert np.all(err <= tol), "train_sum error %g > tol %g at %s" % (
            err.flat[worst], tol.flat[worst], np.unravel_index(worst, err.shape))
        with np.errstate(divide="ignore", invalid="ignore"):
            rel = np.where(st_o != 0, err / np.abs(st_o), 0.0)
        out["max_rel"] = float(rel.max())
    if thr is not None:
        fin = np.isfinite(thr_o)
        assert np.array_equal(np.isfinite(thr), fin)
        if form in ("tiled", "direct"):
            np.testing.assert_allclose(thr[fin], thr_o[fin], rtol=2e-6, atol=0)
    return out


def check_cells(x_np, window, rows, cols, mask_vals, st_vals=None, form="tiled", s_total=None):
    """Compare sampled cells against the oracle's direct CA-CFAR."""
    gr, gf, tr, tf, pfa = window
    m_o, st_o, nt_o, thr_o = oracle.cfar2d_cells(x_np, gr, gf, tr, tf, pfa, rows, cols)
    xv = np.asarray(x_np[rows, cols], dtype=np.float64)
    near = oracle.near_threshold(xv, thr_o, MARGIN)
    bad = (mask_vals != m_o) & ~near
    assert not bad.any(), "sampled mask mismatch at %d cells, first %s" % (
        int(bad.sum()), list(zip(rows[bad][:5], cols[bad][:5])))
    out = {"near": int(near.sum()), "max_rel": 0.0, "n": int(len(rows))}
    if st_vals is not None:
        err = np.abs(st_vals - st_o)
        if form in ("tiled", "direct"):
            tol = TILED_REL * np.abs(st_o)
        else:
            tol = 64 * EPS64 * s_total + 1e-12 * np.abs(st_o)
        tol = np.maximum(tol, 1e-300)
        assert np.all(err <= tol), "sampled train_sum error %g" % float((err / np.maximum(np.abs(st_o), 1e-300)).max())
        out["max_rel"] = float((err / np.maximum(np.abs(st_o), 1e-300)).max())
    return out


def sample_cells(R, F, h_r, h_f, targets=None, n_random=20000, seed=0):
    """Random interior cells, cells in every border band, corners and the
    3x3 neighbourhoods of the planted targets."""
    rng = np.random.default_rng(seed)
    rows = [rng.integers(0, R, n_random)]
    cols = [rng.integers(0, F, n_random)]
    nb = 2000
    for band_r in (np.arange(0, min(R, h_r + 1)), np.arange(max(0, R - h_r - 1), R)):
        rows.append(rng.choice(band_r, nb))
        cols.append(rng.integers(0, F, nb))
    for band_f in (np.arange(0, min(F, h_f + 1)), np.arange(max(0, F - h_f - 1), F)):
        rows.append(rng.integers(0, R, nb))
        cols.append(rng.choice(band_f, nb))
    rows.append(np.array([0, 0, R - 1, R - 1]))
    cols.append(np.array([0, F - 1, 0, F - 1]))
    if targets is not None and len(targets):
        for t in targets:
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    a, b = int(t[0]) + di, int(t[1]) + dj
                    if 0 <= a < R and 0 <= b < F:
                        rows.append(np.array([a]))
                        cols.append(np.array([b]))
    return np.concatenate(rows).astype(np.int64), np.concatenate(cols).astype(np.int64)


def decode_tiled_sat(buf, rows, cols):
    """S(i,j) from the bytes of sat2d's TILED layout (as its declaration in
    include/cfar2d.h describes it), in FP64 on the host: FP32 local sums of
    32 x 32 tiles, FP64 row lines every 32 rows and FP64 column lines every
    32 columns, each region starting at a 256-byte boundary."""
    line = 32

    def up(v):
        return (v + 255) // 256 * 256

    raw = np.ascontiguousarray(buf).view(np.uint8)
    n_i, n_j = (rows + line - 1) // line, (cols + line - 1) // line
    loc_b, row_b = up(rows * cols * 4), up(n_i * cols * 8)
    loc = raw[:rows * cols * 4].view(np.float32).reshape(rows, cols).astype(np.float64)
    rowline = raw[loc_b:loc_b + n_i * cols * 8].view(np.float64).reshape(n_i, cols)
    colline = raw[loc_b + row_b:loc_b + row_b + n_j * rows * 8].view(np.float64).reshape(n_j, rows)
    ti = np.arange(rows) // line
    tj = np.arange(cols) // line
    top = rowline[ti, :]                           # S(32 I - 1, j)
    left = colline[tj, :].T                        # S(i, 32 J - 1)
    cj = np.maximum(tj * line - 1, 0)
    corner = rowline[ti][:, cj] * (tj > 0)[None, :]  # S(32 I - 1, 32 J - 1)
    return top + left - corner + loc
