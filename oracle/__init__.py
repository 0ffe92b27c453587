"""FP64 CPU oracle for integral-image 2D CA-CFAR (arXiv 2012.11077, Sec. II.B).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2012_11077_amd``) never imports it, and the two share no code.

The arithmetic lives in ``cfar_oracle.c`` (plain C, double precision, no FMA);
this module only builds it with gcc and marshals numpy arrays through ctypes.

Functions and the passage each one follows:

* :func:`sat` -- eq. (3), the integral image with a zero leading row/column.
* :func:`cfar2d` -- eqs. (1)-(4): II CA-CFAR over a whole map.
* :func:`cfar2d_cells` -- the direct CA-CFAR of Table I (no integral image),
  on a list of cells; used for sampled checks of large maps.
* :func:`alpha` -- eq. (2), the scale factor, exponent read as -1/N.
* :func:`detection_list` -- the H1 cells of eq. (1) as records in row-major
  order (row, col, CUT, T).
* :func:`pack_mask` -- the mask as bits, 32 cells per word, cell 32 w + u at
  bit u of word w.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cfar_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile ``cfar_oracle.c`` into ``liboracle.so`` with gcc (-O2, no FMA
    contraction; OpenMP only splits the rows of the per-cell loop)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_sat.argtypes = [_vp, _i64, _i64, _i64, _vp]
        lib.oracle_sat.restype = None
        lib.oracle_alpha.argtypes = [_i64, _dbl]
        lib.oracle_alpha.restype = _dbl
        lib.oracle_cfar2d.argtypes = [_vp, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _dbl,
                                      _vp, _vp, _vp, _vp, ctypes.c_int]
        lib.oracle_cfar2d.restype = ctypes.c_int
        lib.oracle_cfar2d_cells.argtypes = [_vp, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _dbl,
                                            _vp, _vp, _i64, _vp, _vp, _vp, _vp]
        lib.oracle_cfar2d_cells.restype = None
        _lib = lib
    return _lib


def _as_f64(x: np.ndarray) -> np.ndarray:
    """Promote a 2D map to C-contiguous float64 (exact for float32 input)."""
    x = np.asarray(x)
    if x.ndim != 2:
        raise ValueError("map must be 2D")
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_vp)


def sat(x: np.ndarray) -> np.ndarray:
    """eq. (3): integral image of ``x`` as an (R+1) x (F+1) float64 array whose
    first row and column are the implied zero boundary."""
    x = _as_f64(x)
    R, F = x.shape
    S = np.empty((R + 1, F + 1), dtype=np.float64)
    _load().oracle_sat(_ptr(x), R, F, F, _ptr(S))
    return S


def alpha(n: int, pfa: float) -> float:
    """eq. (2) scale factor for ``n`` training cells: n * expm1(-ln(pfa)/n)."""
    return float(_load().oracle_alpha(int(n), float(pfa)))


def cfar2d(x: np.ndarray, guard_r: int, guard_f: int, train_r: int, train_f: int, pfa: float,
           threads: int = 1, counts: bool = True):
    """II CA-CFAR (eqs. 1-4) over the whole map.

    Returns ``(mask uint8, train_sum f64, n_train i64, threshold f64)``, each R x F.
    Windows are clipped at the border and the threshold uses the number of
    training cells inside the map.  ``threads`` > 1 runs the per-cell loop on
    that many threads (same outputs); ``counts=False`` skips the training
    counts (``n_train`` is then None), to save memory on large maps.
    """
    x = _as_f64(x)
    R, F = x.shape
    mask = np.empty((R, F), dtype=np.uint8)
    st = np.empty((R, F), dtype=np.float64)
    nt = np.empty((R, F), dtype=np.int64) if counts else None
    thr = np.empty((R, F), dtype=np.float64)
    rc = _load().oracle_cfar2d(_ptr(x), R, F, F, guard_r, guard_f, train_r, train_f, float(pfa),
                               _ptr(mask), _ptr(st), _ptr(nt) if counts else None, _ptr(thr), int(threads))
    if rc != 0:
        raise MemoryError("oracle could not allocate the integral image")
    return mask, st, nt, thr


def cfar2d_cells(x: np.ndarray, guard_r: int, guard_f: int, train_r: int, train_f: int, pfa: float,
                 rows, cols):
    """Direct CA-CFAR (Table I, no integral image) on the listed cells.

    Returns ``(mask, train_sum, n_train, threshold)`` as 1D arrays, one entry per cell.
    """
    x = _as_f64(x) if x.dtype != np.float64 or not x.flags.c_contiguous else x
    R, F = x.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    n = rows.size
    if cols.size != n:
        raise ValueError("rows and cols differ in length")
    if n and (rows.min() < 0 or rows.max() >= R or cols.min() < 0 or cols.max() >= F):
        raise ValueError("cell outside the map")
    mask = np.empty(n, dtype=np.uint8)
    st = np.empty(n, dtype=np.float64)
    nt = np.empty(n, dtype=np.int64)
    thr = np.empty(n, dtype=np.float64)
    _load().oracle_cfar2d_cells(_ptr(x), R, F, F, guard_r, guard_f, train_r, train_f, float(pfa),
                                _ptr(rows), _ptr(cols), n, _ptr(mask), _ptr(st), _ptr(nt), _ptr(thr))
    return mask, st, nt, thr


def near_threshold(x: np.ndarray, thr: np.ndarray, rel: float = 1e-5) -> np.ndarray:
    """Cells whose value lies within ``rel`` (relative) of the oracle threshold.

    Both decisions are acceptable there; parity excludes and counts them.
    """
    xd = np.asarray(x, dtype=np.float64)
    t = np.asarray(thr, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        return np.isfinite(t) & (np.abs(xd - t) <= rel * np.abs(t))


def detection_list(mask: np.ndarray, x: np.ndarray, thr=None):
    """Records of the cells with a nonzero mask, rows outer, columns inner:
    (row, col, X(row, col), T(row, col) or NaN)."""
    out = []
    R, F = mask.shape
    for i in range(R):
        for j in range(F):
            if mask[i, j]:
                out.append((i, j, float(x[i, j]), float(thr[i, j]) if thr is not None else float("nan")))
    return out


def pack_mask(mask: np.ndarray) -> np.ndarray:
    """uint32 words, rows x ceil(F/32): bit u of word w is cell (r, 32 w + u)."""
    R, F = mask.shape
    words = (F + 31) // 32
    out = np.zeros((R, words), dtype=np.uint32)
    for i in range(R):
        for j in range(F):
            if mask[i, j]:
                out[i, j // 32] |= np.uint32(1) << np.uint32(j % 32)
    return out
