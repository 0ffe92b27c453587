"""The C ABI without a GPU: the library loads, exports every function that
include/cfar2d.h declares, and its argument checks, sizing functions, tile
planner and plan-table parser behave as documented (none of these touch the
device)."""
import ctypes
import os
import re

import pytest

from paper_2012_11077_amd import build as hipbuild
from paper_2012_11077_amd import cfar2d as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfar2d.h")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(C.LIB_PATH):
        hipbuild.build()
    return C.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for n in ("sat2d", "cfar2d", "cfar2d_batched", "cfar_submit", "cfar_poll", "cfar_server_create",
              "cfar_server_destroy", "cfar_workspace_bytes", "cfar_plan_for", "cfar_last_error",
              "cfar_detections", "cfar_detections_workspace_bytes", "cfar_mask_pack", "cfar_map_build",
              "cfar_map_bins", "cfar_map_build_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_function(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def _map(rows=100, cols=200, dtype=C.F32, win=(1, 2, 4, 8, 1e-4), x=0x1000, mask=0x2000, ld=None, ldm=None):
    return C.Map(x, dtype, 0, rows, cols, ld or cols, C.make_window(*win), mask, ldm or cols, None, None)


@pytest.mark.parametrize("bad, what", [
    (dict(rows=0), "rows"), (dict(cols=-3), "cols"), (dict(ld=10), "ld < cols"), (dict(ldm=5), "ld_mask"),
    (dict(x=0), "x is NULL"), (dict(mask=0), "mask is NULL"), (dict(dtype=7), "dtype"),
    (dict(win=(1, 1, 0, 0, 1e-3)), "no training"), (dict(win=(1, 1, 2, 2, 1.0)), "pfa"),
    (dict(win=(1, 1, 2, 2, 0.0)), "pfa"), (dict(win=(-1, 1, 2, 2, 1e-3)), "negative"),
    (dict(win=(1, 10, 2, 240, 1e-3)), "TILED form supports"),
])
def test_invalid_maps_are_rejected_before_any_device_work(L, bad, what):
    m = _map(**bad)
    rc = L.cfar2d(ctypes.byref(m), C.TILED, None, 0, None)
    assert rc == C.CFAR_EINVAL
    assert what in C.last_error()
    assert L.cfar_workspace_bytes(ctypes.byref(m), 1, C.TILED) == 0


def test_direct_form_limits(L):
    """DIRECT stages a 4 x 64 tile and its window halo in 64 KiB of LDS:
    wider windows are refused before any device work; its workspace is the
    threshold table only; sat2d does not take it."""
    m = _map(win=(8, 8, 12, 12, 1e-4))
    need = L.cfar_workspace_bytes(ctypes.byref(m), 1, C.DIRECT)
    n_full = 41 * 41 - 17 * 17
    assert need == ((n_full + 1) * 8 + 255) // 256 * 256      # the table beta(0 .. n_full)
    m = _map(dtype=C.F64, win=(4, 4, 24, 24, 1e-4))            # (4+56) x (64+56) x 8 = 57600: fits
    assert L.cfar_workspace_bytes(ctypes.byref(m), 1, C.DIRECT) > 0
    m = _map(win=(1, 2, 4, 200, 1e-4))                          # (4+10) x (64+404) x 4 = 26208: fits
    assert L.cfar_workspace_bytes(ctypes.byref(m), 1, C.DIRECT) > 0
    m = _map(dtype=C.F64, win=(4, 4, 30, 30, 1e-4))             # (4+68) x (64+68) x 8 = 76032: too wide
    assert L.cfar2d(ctypes.byref(m), C.DIRECT, 0x3000, 1 << 20, None) == C.CFAR_EINVAL
    assert "DIRECT form supports" in C.last_error()
    assert L.cfar_workspace_bytes(ctypes.byref(m), 1, C.DIRECT) == 0
    assert L.sat2d_bytes(10, 10, C.DIRECT) == 0
    assert L.sat2d(0x1000, C.F32, 10, 10, 10, C.DIRECT, 0x2000, 1 << 20, 0x3000, 1 << 20, None) == C.CFAR_EINVAL
    ms = (C.Map * 2)(_map(), _map())
    assert L.cfar2d_batched(ms, 2, C.DIRECT, 0, 0x3000, 16, None) == C.CFAR_ENOSPC


def test_detection_argument_checks(L):
    m = _map(rows=10, cols=9000)
    need = L.cfar_detections_workspace_bytes(ctypes.byref(m))
    nb = 10 * 3                                     # 4096 columns per block
    assert need == (nb * 4 + 255) // 256 * 256 + (nb * 8 + 255) // 256 * 256
    assert L.cfar_detections(ctypes.byref(m), None, 5, 0x4000, 0x3000, need, None) == C.CFAR_EINVAL   # out NULL
    assert L.cfar_detections(ctypes.byref(m), 0x5000, -1, 0x4000, 0x3000, need, None) == C.CFAR_EINVAL
    assert L.cfar_detections(ctypes.byref(m), None, 0, None, 0x3000, need, None) == C.CFAR_EINVAL     # count NULL
    assert L.cfar_detections(ctypes.byref(m), None, 0, 0x4000, 0x3000, need - 1, None) == C.CFAR_ENOSPC
    assert L.cfar_mask_pack(ctypes.byref(m), 0x5000, 281, None) == C.CFAR_EINVAL                    # < ceil(9000/32)
    assert L.cfar_mask_pack(ctypes.byref(m), None, 282, None) == C.CFAR_EINVAL
    bad = _map(rows=0)
    assert L.cfar_detections_workspace_bytes(ctypes.byref(bad)) == 0


def test_map_build_argument_checks(L):
    P = C.MapBuildParams
    k0, nb = ctypes.c_int32(), ctypes.c_int32()
    assert L.cfar_map_bins(600, ctypes.byref(P(20.0, 0.3, 0.8, 5, C.F32)), ctypes.byref(k0), ctypes.byref(nb)) == 0
    assert (k0.value, nb.value) == (9, 16)                 # bins 9..24 of 600 traces at 20 Hz
    for p, n in ((P(0.0, 0.3, 0.8, 5, 0), 600), (P(20.0, 0.9, 0.8, 5, 0), 600), (P(20.0, 0.31, 0.32, 5, 0), 600),
                 (P(20.0, 0.3, 0.8, 5, 0), 4001), (P(20.0, 0.3, 0.8, 5, 0), 0)):
        assert L.cfar_map_bins(n, ctypes.byref(p), ctypes.byref(k0), ctypes.byref(nb)) == C.CFAR_EINVAL
        assert L.cfar_map_build_workspace_bytes(n, 1024, ctypes.byref(p)) == 0
    good = P(20.0, 0.3, 0.8, 5, C.F32)
    need = L.cfar_map_build_workspace_bytes(600, 1024, ctypes.byref(good))
    assert need >= 600 * 1024 * 8
    for p in (P(20.0, 0.3, 0.8, 4, 0), P(20.0, 0.3, 0.8, 1025, 0), P(20.0, 0.3, 0.8, 5, 7)):   # even / long L, dtype
        assert L.cfar_map_build(0x1000, C.F32, 600, 1024, 1024, ctypes.byref(p), 0x2000, 16, 0x3000, need,
                                None) == C.CFAR_EINVAL
    assert L.cfar_map_build(0x1000, C.F32, 600, 1024, 1000, ctypes.byref(good), 0x2000, 16, 0x3000, need,
                            None) == C.CFAR_EINVAL           # ld_raw < n_samples
    assert L.cfar_map_build(0x1000, C.F32, 600, 1024, 1024, ctypes.byref(good), 0x2000, 15, 0x3000, need,
                            None) == C.CFAR_EINVAL           # ld_map < bins
    assert L.cfar_map_build(0x1000, C.F32, 600, 1024, 1024, ctypes.byref(good), 0x2000, 16, 0x3000, need - 1,
                            None) == C.CFAR_ENOSPC


def test_workspace_too_small_is_enospc(L):
    m = _map()
    need = L.cfar_workspace_bytes(ctypes.byref(m), 1, C.TILED)
    assert need > 0
    assert L.cfar2d(ctypes.byref(m), C.TILED, 0x3000, 16, None) == C.CFAR_ENOSPC
    assert L.cfar2d(ctypes.byref(m), C.PLAIN, 0x3000, 16, None) == C.CFAR_ENOSPC
    ms = (C.Map * 2)(m, m)
    assert L.cfar2d_batched(ms, 2, C.TILED, 0, 0x3000, 16, None) == C.CFAR_ENOSPC
    need_plain = L.cfar_workspace_bytes(ctypes.byref(m), 1, C.PLAIN)
    assert need_plain >= 100 * 200 * 8   # the FP64 integral image itself


def test_sat2d_sizes(L):
    assert L.sat2d_bytes(3, 5, C.PLAIN) == 3 * 5 * 8
    assert L.sat2d_bytes(0, 5, C.PLAIN) == 0 or L.sat2d_bytes(0, 5, C.PLAIN) >= 0
    assert L.sat2d_workspace_bytes(1000, 1000, C.PLAIN) > 0


@pytest.fixture
def builtin_model(L):
    """The built-in cost model for the test; the package's plan table (if
    any) is loaded again afterwards."""
    C.plan_load(None)
    yield
    if os.path.exists(C.DEFAULT_PLAN_TABLE) and os.environ.get("CFAR2D_PLAN_TABLE") is None:
        C.plan_load(C.DEFAULT_PLAN_TABLE)


def test_planner_follows_the_cost_model(L, builtin_model):
    def plan(rows, cols, win):
        m = _map(rows, cols, win=win)
        p = C.Plan()
        assert L.cfar_plan_for(ctypes.byref(m), ctypes.byref(p)) == C.CFAR_OK
        return p.k_cols, p.rows_per_unit, p.ring_bytes
    assert plan(16384, 16384, (4, 4, 24, 24, 1e-5))[0] == 4      # wide map: k = 4
    assert plan(16384, 16384, (1, 1, 1, 1, 1e-5))[0] == 4
    assert plan(300, 65, (1, 1, 4, 4, 1e-3))[0] == 2             # narrow map: k = 2
    k, rs, ring = plan(50, 40000, (1, 1, 4, 4, 1e-3))
    assert rs == 50 and ring == -1                                # short wide map: one row chunk
    # few units at 128 rows (8 row chunks x 3 strips): shorter units, so that
    # the map spreads over at least 128 of them
    assert plan(1024, 600, (4, 4, 8, 8, 1e-4)) == (4, 24, -1)
    assert plan(50, 4000, (1, 1, 4, 4, 1e-3))[1] == 16            # not below 16 rows


def test_plan_table_rules(L, tmp_path, builtin_model):
    good = tmp_path / "plans.txt"
    good.write_text("# dtype cols rows hf hr k rs [ring]\n"
                    "f32 0 1000 0 100000 0 300 0 300 8 32 4096\n"
                    "any 0 100000000 0 100000000 0 300 0 300 2 128\n")
    try:
        C.plan_load(str(good))
        m = _map(100, 500)
        p = C.Plan()
        assert L.cfar_plan_for(ctypes.byref(m), ctypes.byref(p)) == 0
        assert (p.k_cols, p.rows_per_unit, p.ring_bytes) == (8, 32, 4096)
        m = _map(100, 5000)
        assert L.cfar_plan_for(ctypes.byref(m), ctypes.byref(p)) == 0
        assert (p.k_cols, p.rows_per_unit, p.ring_bytes) == (2, 100, -1)   # rows_per_unit capped at rows
        bad = tmp_path / "bad.txt"
        bad.write_text("f32 0 1 0 1 0 1 0 1 3 64\n")
        with pytest.raises(C.CfarError):
            C.plan_load(str(bad))
        bad.write_text("f16 0 1 0 1 0 1 0 1 4 64\n")
        with pytest.raises(C.CfarError):
            C.plan_load(str(bad))
    finally:
        C.plan_load(None)


def test_package_plan_table_parses(L):
    if os.path.exists(C.DEFAULT_PLAN_TABLE):
        C.plan_load(C.DEFAULT_PLAN_TABLE)


def test_invalid_plans_are_rejected(L):
    m = _map()
    for p in (C.Plan(3, 64, -1), C.Plan(4, 0, -1), C.Plan(4, 64, -2), C.Plan(4, 64, 70000)):
        assert L.cfar2d_with_plan(ctypes.byref(m), ctypes.byref(p), 0x3000, 1 << 20, None) == C.CFAR_EINVAL


def test_server_argument_checks(L):
    h = ctypes.c_void_p()
    assert L.cfar_server_create(None, ctypes.byref(h)) == C.CFAR_EINVAL
    for opts in (C.ServerOpts(1 << 30, 0, 2, 8, 4), C.ServerOpts(1 << 30, 8, 0, 8, 4),
                 C.ServerOpts(1 << 30, 8, 17, 8, 4), C.ServerOpts(1 << 30, 8, 2, 0, 4),
                 C.ServerOpts(1 << 30, 8, 2, 8, 0), C.ServerOpts(1000, 8, 2, 8, 4)):
        assert L.cfar_server_create(ctypes.byref(opts), ctypes.byref(h)) == C.CFAR_EINVAL
    t = ctypes.c_uint64()
    m = _map()
    assert L.cfar_submit(None, ctypes.byref(m), 1, 0, ctypes.byref(t)) == C.CFAR_EINVAL
    n = ctypes.c_int32()
    assert L.cfar_poll(None, None, 4, 0, ctypes.byref(n)) == C.CFAR_EINVAL
    assert L.cfar_server_shutdown(None, 1) == C.CFAR_EINVAL
    assert L.cfar_server_destroy(None) == C.CFAR_EINVAL


def test_version_and_timing_errors(L):
    assert C.version()
    v = ctypes.c_double()
    assert L.cfar_timing_read(None) == C.CFAR_EINVAL
    assert L.cfar_timing_read(ctypes.byref(v)) == C.CFAR_EINVAL   # nothing timed on this thread
