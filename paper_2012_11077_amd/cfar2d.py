"""ctypes binding of libcfar2d.so (C ABI in include/cfar2d.h).

Argument marshalling only: every step of the detector runs in the library's
HIP kernels.  PyTorch provides device memory and streams; tensors are passed
by their data pointers.  If the library is not built, every call raises.

Functions follow the C names: :func:`sat2d`, :func:`cfar2d`,
:func:`cfar2d_batched`, :func:`workspace_bytes`, :func:`plan_for`,
:func:`plan_load`, :func:`cfar2d_with_plan`, and the streaming server
:class:`Server` (``cfar_server_create`` / ``cfar_submit`` / ``cfar_poll`` /
``cfar_server_shutdown`` / ``cfar_server_destroy``).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcfar2d.so")
# Tile-plan table written by the autotuner (paper_2012_11077_amd/autotune.py);
# CFAR2D_PLAN_TABLE overrides it ("" = the library's built-in cost model).
DEFAULT_PLAN_TABLE = os.path.join(_PKG, "plan_table.txt")

CFAR_OK, CFAR_EINVAL, CFAR_ENOSPC, CFAR_EDEVICE, CFAR_EAGAIN, CFAR_ESHUTDOWN = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
PLAIN, TILED, DIRECT = 0, 1, 2
BATCH_GRAPH = 1
SUBMIT_HOST, SUBMIT_PACKED_MASK = 1, 2
STATUS_NAMES = {0: "CFAR_OK", -1: "CFAR_EINVAL", -2: "CFAR_ENOSPC", -3: "CFAR_EDEVICE",
                -4: "CFAR_EAGAIN", -5: "CFAR_ESHUTDOWN"}


class CfarError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


class Window(ctypes.Structure):
    _fields_ = [("guard_r", ctypes.c_int32), ("guard_f", ctypes.c_int32),
                ("train_r", ctypes.c_int32), ("train_f", ctypes.c_int32), ("pfa", ctypes.c_double)]


class MapBuildParams(ctypes.Structure):
    _fields_ = [("fs_slow", ctypes.c_double), ("f_lo", ctypes.c_double), ("f_hi", ctypes.c_double),
                ("mean_len", ctypes.c_int32), ("out_dtype", ctypes.c_int32)]


class Map(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("win", Window), ("mask", ctypes.c_void_p), ("ld_mask", ctypes.c_int64),
                ("train_sum", ctypes.c_void_p), ("threshold", ctypes.c_void_p)]


class Plan(ctypes.Structure):
    _fields_ = [("k_cols", ctypes.c_int32), ("rows_per_unit", ctypes.c_int32), ("ring_bytes", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device_budget_bytes", ctypes.c_size_t), ("max_inflight_frames", ctypes.c_int32),
                ("n_hip_streams", ctypes.c_int32), ("queue_depth", ctypes.c_int32),
                ("max_batch_frames", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("user_tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("device_bytes_in_use", ctypes.c_size_t), ("device_bytes_peak", ctypes.c_size_t),
                ("inflight_frames", ctypes.c_int32), ("queued_frames", ctypes.c_int32)]


_lib = None
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_PMap = ctypes.POINTER(Map)


def lib():
    """Load libcfar2d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcfar2d.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.cfar_last_error.restype = ctypes.c_char_p
        L.cfar_version.restype = ctypes.c_char_p
        L.sat2d_bytes.argtypes = [_i64, _i64, _i32]
        L.sat2d_bytes.restype = _sz
        L.sat2d_workspace_bytes.argtypes = [_i64, _i64, _i32]
        L.sat2d_workspace_bytes.restype = _sz
        L.sat2d.argtypes = [_vp, _i32, _i64, _i64, _i64, _i32, _vp, _sz, _vp, _sz, _vp]
        L.cfar_workspace_bytes.argtypes = [_PMap, _i32, _i32]
        L.cfar_workspace_bytes.restype = _sz
        L.cfar2d.argtypes = [_PMap, _i32, _vp, _sz, _vp]
        L.cfar2d_batched.argtypes = [_PMap, _i32, _i32, _i32, _vp, _sz, _vp]
        L.cfar2d_static.argtypes = [_PMap, _vp]
        L.cfar2d_static_max_bytes.argtypes = []
        L.cfar2d_static_max_bytes.restype = _sz
        L.cfar_plan_for.argtypes = [_PMap, ctypes.POINTER(Plan)]
        L.cfar_plan_load.argtypes = [ctypes.c_char_p]
        L.cfar2d_with_plan.argtypes = [_PMap, ctypes.POINTER(Plan), _vp, _sz, _vp]
        L.cfar_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(_vp)]
        L.cfar_submit.argtypes = [_vp, _PMap, _i32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        L.cfar_poll.argtypes = [_vp, ctypes.POINTER(Completion), _i32, _i32, ctypes.POINTER(_i32)]
        L.cfar_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
        L.cfar_server_shutdown.argtypes = [_vp, _i32]
        L.cfar_server_destroy.argtypes = [_vp]
        L.cfar_host_alloc.argtypes = [_sz, ctypes.POINTER(_vp)]
        L.cfar_host_free.argtypes = [_vp]
        _PMB = ctypes.POINTER(MapBuildParams)
        L.cfar_map_bins.argtypes = [_i64, _PMB, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
        L.cfar_map_build_workspace_bytes.argtypes = [_i64, _i64, _PMB]
        L.cfar_map_build_workspace_bytes.restype = _sz
        L.cfar_map_build.argtypes = [_vp, _i32, _i64, _i64, _i64, _PMB, _vp, _i64, _vp, _sz, _vp]
        L.cfar_detections_workspace_bytes.argtypes = [_PMap]
        L.cfar_detections_workspace_bytes.restype = _sz
        L.cfar_detections.argtypes = [_PMap, _vp, _i64, _vp, _vp, _sz, _vp]
        L.cfar_mask_pack.argtypes = [_PMap, _vp, _i64, _vp]
        L.cfar_timing_enable.argtypes = [_i32]
        L.cfar_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double)]
        for name in ("sat2d", "cfar2d", "cfar2d_static", "cfar2d_batched", "cfar_plan_for", "cfar_plan_load",
                     "cfar2d_with_plan", "cfar_timing_enable", "cfar_timing_read", "cfar_server_create",
                     "cfar_submit", "cfar_poll", "cfar_server_stats_get", "cfar_server_shutdown",
                     "cfar_server_destroy", "cfar_host_alloc", "cfar_host_free", "cfar_detections",
                     "cfar_mask_pack", "cfar_map_bins", "cfar_map_build"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
        table = os.environ.get("CFAR2D_PLAN_TABLE")
        if table is None and os.path.exists(DEFAULT_PLAN_TABLE):
            table = DEFAULT_PLAN_TABLE
        if table:
            _check(L.cfar_plan_load(table.encode()))
    return _lib


def last_error() -> str:
    return lib().cfar_last_error().decode()


def version() -> str:
    return lib().cfar_version().decode()


def _check(rc: int) -> None:
    if rc != CFAR_OK:
        raise CfarError(rc, last_error())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, int):
        return stream or None
    return stream.cuda_stream or None


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("map must be float32 or float64, got %s" % t.dtype)


def _check_2d(t: torch.Tensor, name: str) -> None:
    if t.dim() != 2:
        raise ValueError("%s must be 2D" % name)
    if t.size(1) > 1 and t.stride(1) != 1:
        raise ValueError("%s must have unit stride along columns" % name)


def make_window(guard_r: int, guard_f: int, train_r: int, train_f: int, pfa: float) -> Window:
    return Window(int(guard_r), int(guard_f), int(train_r), int(train_f), float(pfa))


def make_map(x: torch.Tensor, window, mask: torch.Tensor, train_sum: Optional[torch.Tensor] = None,
             threshold: Optional[torch.Tensor] = None) -> Map:
    """C descriptor of one map.  ``window`` is a :class:`Window` or a tuple
    (guard_r, guard_f, train_r, train_f, pfa).  The mask (uint8) and the
    optional float64 outputs share the mask's leading dimension."""
    _check_2d(x, "x")
    _check_2d(mask, "mask")
    if mask.dtype != torch.uint8:
        raise TypeError("mask must be uint8")
    if tuple(mask.shape) != tuple(x.shape):
        raise ValueError("mask shape differs from the map")
    w = window if isinstance(window, Window) else make_window(*window)
    ldm = mask.stride(0) if mask.size(0) > 1 else mask.size(1)
    for name, t in (("train_sum", train_sum), ("threshold", threshold)):
        if t is not None:
            _check_2d(t, name)
            if t.dtype != torch.float64 or tuple(t.shape) != tuple(x.shape):
                raise ValueError("%s must be float64 with the map's shape" % name)
            if (t.stride(0) if t.size(0) > 1 else t.size(1)) != ldm:
                raise ValueError("%s must share the mask's leading dimension" % name)
    ld = x.stride(0) if x.size(0) > 1 else x.size(1)
    return Map(x.data_ptr(), _dtype_code(x), 0, x.size(0), x.size(1), ld, w, mask.data_ptr(), ldm,
               train_sum.data_ptr() if train_sum is not None else None,
               threshold.data_ptr() if threshold is not None else None)


def _alloc_ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def sat2d(x: torch.Tensor, form: int = PLAIN, out: Optional[torch.Tensor] = None,
          ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Integral image (eq. 3) of ``x``.  PLAIN: returns an R x F float64
    tensor.  TILED: returns the raw byte buffer of the tiled layout (see
    include/cfar2d.h)."""
    _check_2d(x, "x")
    L = lib()
    R, F = x.shape
    nbytes = L.sat2d_bytes(R, F, form)
    if nbytes == 0:
        raise CfarError(CFAR_EINVAL, "invalid shape or form")
    if out is None:
        out = (torch.empty((R, F), dtype=torch.float64, device=x.device) if form == PLAIN
               else torch.empty(nbytes, dtype=torch.uint8, device=x.device))
    if ws is None:
        ws = _alloc_ws(L.sat2d_workspace_bytes(R, F, form), x.device)
    ld = x.stride(0) if R > 1 else F
    _check(L.sat2d(x.data_ptr(), _dtype_code(x), R, F, ld, form, out.data_ptr(),
                   out.numel() * out.element_size(), ws.data_ptr(), ws.numel(),
                   _stream_handle(stream)))
    return out


def workspace_bytes(maps: Sequence[Map], form: int) -> int:
    arr = (Map * len(maps))(*maps)
    n = lib().cfar_workspace_bytes(arr, len(maps), form)
    if n == 0:
        raise CfarError(CFAR_EINVAL, last_error())
    return int(n)


def cfar2d(x: torch.Tensor, window, form: int = TILED, mask: Optional[torch.Tensor] = None,
           train_sum: Optional[torch.Tensor] = None, threshold: Optional[torch.Tensor] = None,
           ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """CA-CFAR over one map (eqs. 1-4); returns the uint8 mask."""
    if mask is None:
        mask = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    m = make_map(x, window, mask, train_sum, threshold)
    if ws is None:
        ws = _alloc_ws(workspace_bytes([m], form), x.device)
    _check(lib().cfar2d(ctypes.byref(m), form, ws.data_ptr(), ws.numel(), _stream_handle(stream)))
    return mask


def cfar2d_static(x: torch.Tensor, window, mask: torch.Tensor, train_sum: Optional[torch.Tensor] = None,
                  threshold: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """TILED CA-CFAR over one map with the library's static device workspace
    (allocates nothing; the caller passes the outputs)."""
    m = make_map(x, window, mask, train_sum, threshold)
    _check(lib().cfar2d_static(ctypes.byref(m), _stream_handle(stream)))
    return mask


def cfar2d_with_plan(x: torch.Tensor, window, k_cols: int, rows_per_unit: int,
                     mask: Optional[torch.Tensor] = None, train_sum=None, threshold=None,
                     ws: Optional[torch.Tensor] = None, stream=None, ring_bytes: int = -1) -> torch.Tensor:
    """TILED CA-CFAR with an explicit tile plan (autotuner probe); ring_bytes
    -1 takes the library default."""
    if mask is None:
        mask = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    m = make_map(x, window, mask, train_sum, threshold)
    if ws is None:
        ws = _alloc_ws(workspace_bytes([m], TILED), x.device)
    p = Plan(int(k_cols), int(rows_per_unit), int(ring_bytes))
    _check(lib().cfar2d_with_plan(ctypes.byref(m), ctypes.byref(p), ws.data_ptr(), ws.numel(),
                                  _stream_handle(stream)))
    return mask


class Batch:
    """A prepared batch: the C descriptor array plus a workspace, reusable
    across calls on the same tensors (what a serving loop or benchmark does)."""

    def __init__(self, xs: Sequence[torch.Tensor], windows: Sequence, form: int = TILED,
                 masks: Optional[Sequence[torch.Tensor]] = None, train_sums=None, thresholds=None,
                 ws: Optional[torch.Tensor] = None):
        n = len(xs)
        if n == 0:
            raise ValueError("empty batch")
        if masks is None:
            masks = [torch.empty(x.shape, dtype=torch.uint8, device=x.device) for x in xs]
        self.xs, self.masks, self.form = list(xs), list(masks), form
        ts = train_sums or [None] * n
        th = thresholds or [None] * n
        self.maps = (Map * n)(*[make_map(xs[i], windows[i], masks[i], ts[i], th[i]) for i in range(n)])
        need = lib().cfar_workspace_bytes(self.maps, n, form)
        if need == 0:
            raise CfarError(CFAR_EINVAL, last_error())
        self.ws = ws if ws is not None else _alloc_ws(need, xs[0].device)
        if self.ws.numel() < need:
            raise CfarError(CFAR_ENOSPC, "workspace too small")

    def run(self, flags: int = BATCH_GRAPH, stream=None) -> List[torch.Tensor]:
        _check(lib().cfar2d_batched(self.maps, len(self.xs), self.form, flags, self.ws.data_ptr(),
                                    self.ws.numel(), _stream_handle(stream)))
        return self.masks


def cfar2d_batched(xs: Sequence[torch.Tensor], windows: Sequence, form: int = TILED,
                   masks=None, train_sums=None, thresholds=None, flags: int = BATCH_GRAPH,
                   ws: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """CA-CFAR over many maps (own sizes, windows and Pfa) in one call."""
    b = Batch(xs, windows, form, masks, train_sums, thresholds, ws)
    return b.run(flags, stream)


def plan_for(x: torch.Tensor, window) -> Tuple[int, int, int]:
    """(k_cols, rows_per_unit, ring_bytes) the TILED form uses for this map."""
    m = make_map(x, window, _mask_like(x))
    p = Plan()
    _check(lib().cfar_plan_for(ctypes.byref(m), ctypes.byref(p)))
    return int(p.k_cols), int(p.rows_per_unit), int(p.ring_bytes)


def _mask_like(x: torch.Tensor) -> torch.Tensor:
    return torch.empty(x.shape, dtype=torch.uint8, device=x.device)


def map_bins(n_traces: int, fs_slow: float, f_lo: float = 0.3, f_hi: float = 0.8) -> Tuple[int, int]:
    """(first DFT bin, number of bins) the band keeps for n_traces traces."""
    p = MapBuildParams(float(fs_slow), float(f_lo), float(f_hi), 1, F32)
    k0, nb = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().cfar_map_bins(int(n_traces), ctypes.byref(p), ctypes.byref(k0), ctypes.byref(nb)))
    return int(k0.value), int(nb.value)


def build_map(raw: torch.Tensor, fs_slow: float, f_lo: float = 0.3, f_hi: float = 0.8, mean_len: int = 5,
              out_dtype=torch.float32, stream=None) -> torch.Tensor:
    """Range x slow-time-frequency power map (Sec. II.A) of a raw record
    ``raw`` (n_traces x n_samples, one trace per row, on the device)."""
    _check_2d(raw, "raw")
    N, M = raw.shape
    p = MapBuildParams(float(fs_slow), float(f_lo), float(f_hi), int(mean_len),
                       F32 if out_dtype == torch.float32 else F64)
    _, nb = map_bins(N, fs_slow, f_lo, f_hi)
    out = torch.empty((M, nb), dtype=out_dtype, device=raw.device)
    need = lib().cfar_map_build_workspace_bytes(N, M, ctypes.byref(p))
    if need == 0:
        raise CfarError(CFAR_EINVAL, last_error())
    ws = _alloc_ws(need, raw.device)
    ld = raw.stride(0) if N > 1 else M
    _check(lib().cfar_map_build(raw.data_ptr(), _dtype_code(raw), N, M, ld, ctypes.byref(p), out.data_ptr(), nb,
                                ws.data_ptr(), ws.numel(), _stream_handle(stream)))
    return out


DETECTION_BYTES = 24   # cfar_detection: int32 row, int32 col, float64 cut, float64 threshold


def detections(x: torch.Tensor, mask: torch.Tensor, threshold: Optional[torch.Tensor] = None,
               capacity: Optional[int] = None, stream=None):
    """Detections of a map whose mask the detector wrote (same stream): a dict
    of device tensors ``row``, ``col`` (int32), ``cut``, ``threshold``
    (float64; NaN without a threshold output), in row-major order of the
    cells, and ``count`` (the total, which may exceed ``capacity``).  With
    no capacity given the count is taken first (one synchronisation) and
    the list sized to it."""
    m = make_map(x, (0, 0, 0, 1, 0.5), mask, None, threshold)
    cnt = torch.zeros(1, dtype=torch.int64, device=x.device)
    ws = _alloc_ws(lib().cfar_detections_workspace_bytes(ctypes.byref(m)), x.device)
    h = _stream_handle(stream)
    if capacity is None:
        _check(lib().cfar_detections(ctypes.byref(m), None, 0, cnt.data_ptr(), ws.data_ptr(), ws.numel(), h))
        torch.cuda.synchronize(x.device)   # the count was written on the library's stream `h`
        capacity = int(cnt.item())
    cap = int(capacity)
    buf = torch.empty(max(cap, 1) * DETECTION_BYTES // 8, dtype=torch.float64, device=x.device)
    _check(lib().cfar_detections(ctypes.byref(m), buf.data_ptr() if cap > 0 else None, cap, cnt.data_ptr(),
                                 ws.data_ptr(), ws.numel(), h))
    torch.cuda.synchronize(x.device)
    n = min(int(cnt.item()), cap)
    rec = buf.view(-1, 3)[:n]
    rc = rec.view(torch.int32)[:, :2]
    return {"row": rc[:, 0], "col": rc[:, 1], "cut": rec[:, 1], "threshold": rec[:, 2], "count": int(cnt.item())}


def mask_pack(x: torch.Tensor, mask: torch.Tensor, stream=None) -> torch.Tensor:
    """Bit-packed mask: int32 tensor rows x ceil(cols/32); bit u of word w of
    row r is cell (r, 32 w + u)."""
    m = make_map(x, (0, 0, 0, 1, 0.5), mask)
    R, F = mask.shape
    words = (F + 31) // 32
    bits = torch.empty((R, words), dtype=torch.int32, device=x.device)
    _check(lib().cfar_mask_pack(ctypes.byref(m), bits.data_ptr(), words, _stream_handle(stream)))
    return bits


def timing_enable(on: bool) -> None:
    """Record HIP events around the kernels of TILED launches (no graphs meanwhile) and DIRECT launches."""
    _check(lib().cfar_timing_enable(1 if on else 0))


def timing_read() -> float:
    """Kernel milliseconds of the calling thread's last timed TILED or DIRECT launch."""
    v = ctypes.c_double()
    _check(lib().cfar_timing_read(ctypes.byref(v)))
    return v.value


def plan_load(path: Optional[str]) -> None:
    _check(lib().cfar_plan_load(path.encode() if path else None))


def host_empty(shape, dtype=torch.float32) -> torch.Tensor:
    """A CPU tensor in page-locked memory from cfar_host_alloc (full-speed
    copies for frames submitted from host memory); freed when the tensor and
    every view of it are gone."""
    import weakref
    import numpy as np
    np_dtype = {torch.float32: np.float32, torch.float64: np.float64, torch.uint8: np.uint8,
                torch.int32: np.int32}[dtype]
    n = 1
    for d in shape:
        n *= int(d)
    nbytes = max(1, n * np.dtype(np_dtype).itemsize)
    p = ctypes.c_void_p()
    _check(lib().cfar_host_alloc(nbytes, ctypes.byref(p)))
    buf = (ctypes.c_char * nbytes).from_address(p.value)
    arr = np.frombuffer(buf, dtype=np_dtype, count=n).reshape(shape)
    weakref.finalize(buf, lib().cfar_host_free, ctypes.c_void_p(p.value))
    return torch.from_numpy(arr)


class Server:
    """The library's streaming server (continuous batching of frames from
    many streams).  Frames are either device tensors or host tensors (pinned
    memory lets the copies overlap); the caller keeps each frame's tensors
    alive until its ticket completes."""

    def __init__(self, device_budget_bytes: int = 8 << 30, max_inflight_frames: int = 64,
                 n_hip_streams: int = 4, queue_depth: int = 256, max_batch_frames: int = 32):
        o = ServerOpts(int(device_budget_bytes), int(max_inflight_frames), int(n_hip_streams),
                       int(queue_depth), int(max_batch_frames))
        self._h = ctypes.c_void_p()
        _check(lib().cfar_server_create(ctypes.byref(o), ctypes.byref(self._h)))

    def submit(self, x: torch.Tensor, window, mask: torch.Tensor, tag: int = 0, train_sum=None,
               threshold=None) -> Optional[int]:
        """Ticket of the submitted frame, or None when the queue is full
        (CFAR_EAGAIN).  Other errors raise.  A host frame's mask may be an
        int32 tensor of rows x ceil(cols/32) words: it then receives the
        bit-packed mask (cell (r, 32 w + u) at bit u of word w)."""
        on_host = x.device.type == "cpu"
        if (mask.device.type == "cpu") != on_host:
            raise ValueError("x and mask must both be on the host or both on the device")
        if not on_host:
            # the server reads device frames on its own streams: the work that
            # produced this one (on the current stream) must be done first
            torch.cuda.current_stream(x.device).synchronize()
        flags = SUBMIT_HOST if on_host else 0
        if mask.dtype == torch.int32:
            _check_2d(x, "x")
            _check_2d(mask, "mask")
            R, F = x.shape
            if mask.size(0) != R or mask.size(1) < (F + 31) // 32:
                raise ValueError("packed mask must be rows x ceil(cols/32) words")
            w = window if isinstance(window, Window) else make_window(*window)
            m = Map(x.data_ptr(), _dtype_code(x), 0, R, F, x.stride(0) if R > 1 else F, w, mask.data_ptr(),
                    mask.stride(0) if R > 1 else mask.size(1), None, None)
            flags |= SUBMIT_PACKED_MASK
        else:
            m = make_map(x, window, mask, train_sum, threshold)
        t = ctypes.c_uint64()
        rc = lib().cfar_submit(self._h, ctypes.byref(m), flags, int(tag), ctypes.byref(t))
        if rc == CFAR_EAGAIN:
            return None
        _check(rc)
        return int(t.value)

    def poll(self, max_n: int = 64, timeout_us: int = 0) -> List[Completion]:
        buf = (Completion * max_n)()
        n = ctypes.c_int32()
        _check(lib().cfar_poll(self._h, buf, int(max_n), int(timeout_us), ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib().cfar_server_stats_get(self._h, ctypes.byref(st)))
        return st

    def shutdown(self, drain: bool = True) -> None:
        _check(lib().cfar_server_shutdown(self._h, 1 if drain else 0))

    def close(self) -> None:
        if self._h:
            _check(lib().cfar_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
