"""The allocation-free entry point (cfar2d_static) through the C ABI: the
same result as cfar2d in the TILED form, on two calls in a row (the second
on a smaller map, so the static workspace holds the first call's contents),
checked against the oracle; windows too large for the static workspace are
refused."""
import numpy as np
import pytest
import torch

from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import check_full, say

DEV = "cuda:0"


@pytest.mark.gpu
def test_static_equals_cfar2d_twice():
    specs = [synth.MapSpec(900, 1300, "f32", "lognormal", 2.0, n_targets=20, guard_r=4, guard_f=3, train_r=20,
                           train_f=24, pfa=1e-5, seed=(61, 1)),
             synth.MapSpec(257, 301, "f32", "exp", 1.0, n_targets=5, guard_r=1, guard_f=2, train_r=6, train_f=5,
                           pfa=1e-3, seed=(61, 2))]
    stream = torch.cuda.Stream()
    for spec in specs:
        x_np = synth.generate(spec)
        x = torch.from_numpy(x_np).to(DEV)
        R, F = x.shape
        ref_m = C.cfar2d(x, spec.window, C.TILED)
        ref_st = torch.empty((R, F), dtype=torch.float64, device=DEV)
        C.cfar2d(x, spec.window, C.TILED, mask=torch.empty_like(ref_m), train_sum=ref_st)
        torch.cuda.synchronize()
        m = torch.full((R, F), 7, dtype=torch.uint8, device=DEV)
        st = torch.empty((R, F), dtype=torch.float64, device=DEV)
        say("static", R, F, spec.window)
        C.cfar2d_static(x, spec.window, m, stream=stream)
        m2 = torch.full((R, F), 7, dtype=torch.uint8, device=DEV)
        C.cfar2d_static(x, spec.window, m2, train_sum=st, stream=stream)
        stream.synchronize()
        assert torch.equal(m, ref_m)
        assert torch.equal(m2, ref_m)
        assert np.array_equal(st.cpu().numpy().view(np.int64), ref_st.cpu().numpy().view(np.int64))
        check_full(x_np, spec.window, m.cpu().numpy(), st.cpu().numpy(), None, "tiled")


def test_static_refuses_windows_beyond_its_workspace():
    """Validation happens on the host before any device work: a window whose
    threshold table does not fit the static workspace is refused."""
    cap_cells = (C.lib().cfar2d_static_max_bytes() - 256) // 8 - 1
    h = 200  # (2h+1)^2 - 1 training cells
    assert (2 * h + 1) ** 2 - 1 > cap_cells
    m = C.Map(0x1000, 0, 0, 500, 500, 500, C.make_window(0, 0, h, h, 1e-3), 0x1000, 500, None, None)
    rc = C.lib().cfar2d_static(C.ctypes.byref(m), None)
    assert rc == C.CFAR_ENOSPC
    assert b"static workspace" in C.lib().cfar_last_error()
