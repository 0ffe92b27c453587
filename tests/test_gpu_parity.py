"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Sizes the oracle finishes in seconds (several tiles and ragged tails), the
edge cases of the method (1x1 maps, windows wider than the map, zero guard
or zero training on one axis, strided and misaligned maps), and the full
benchmark sizes checked on sampled cells against the oracle's direct sums.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import check_cells, check_full, decode_tiled_sat, sample_cells, say

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FORMS = {"plain": C.PLAIN, "tiled": C.TILED, "direct": C.DIRECT}


def _run(x_np, window, form, with_outputs=True, x_dev=None):
    x = x_dev if x_dev is not None else torch.from_numpy(x_np).to(DEV)
    R, F = x.shape
    mask = torch.empty((R, F), dtype=torch.uint8, device=DEV)
    st = torch.empty((R, F), dtype=torch.float64, device=DEV) if with_outputs else None
    th = torch.empty((R, F), dtype=torch.float64, device=DEV) if with_outputs else None
    C.cfar2d(x, window, FORMS[form], mask=mask, train_sum=st, threshold=th)
    torch.cuda.synchronize()
    return (mask.cpu().numpy(), st.cpu().numpy() if st is not None else None,
            th.cpu().numpy() if th is not None else None)


@pytest.mark.parametrize("form", ["plain", "tiled", "direct"])
def test_config0(form):
    spec = synth.config0()
    x, targets = synth.generate_with_targets(spec)
    say("config0", form, spec.rows, spec.cols)
    mask, st, th = _run(x, spec.window, form)
    r = check_full(x, spec.window, mask, st, th, form)
    say("config0", form, r)
    for t in targets:   # 15 dB targets on Exp(1) clutter are found by both
        assert mask[int(t[0]), int(t[1])] == 1


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("form", ["plain", "tiled", "direct"])
def test_random_small_maps(form, dtype):
    specs = synth.random_small_specs(40, seed=11 if dtype == "f32" else 12, dtype=dtype)
    for k, spec in enumerate(specs):
        x = synth.generate(spec)
        say("random", form, dtype, k, spec.rows, spec.cols, spec.window)
        mask, st, th = _run(x, spec.window, form)
        check_full(x, spec.window, mask, st, th, form)


EDGE = [
    # rows, cols, gr, gf, tr, tf, pfa
    (1, 1, 0, 0, 1, 1, 0.5),
    (1, 300, 0, 2, 3, 9, 1e-2),
    (300, 1, 2, 0, 9, 3, 1e-2),
    (3, 3, 4, 4, 4, 4, 1e-3),
    (5, 700, 1, 1, 0, 6, 1e-3),        # no training along rows
    (700, 5, 1, 1, 6, 0, 1e-3),        # no training along columns
    (97, 131, 0, 0, 5, 5, 1e-4),       # no guard
    (64, 400, 4, 4, 24, 24, 1e-5),
    (40, 1100, 2, 10, 3, 237, 1e-4),   # column half-width at the TILED limit (247)
    (130, 520, 1, 0, 2, 247, 1e-3),    # hf = 247
    (256, 456, 4, 4, 24, 24, 1e-5),    # exactly one strip wide at k = 8
    (513, 457, 3, 3, 16, 16, 1e-6),    # ragged tails
]


@pytest.mark.parametrize("form", ["plain", "tiled", "direct"])
@pytest.mark.parametrize("case", EDGE, ids=[str(c[:2] + c[2:6]) for c in EDGE])
def test_edge_shapes(form, case):
    R, F, gr, gf, tr, tf, pfa = case
    spec = synth.MapSpec(R, F, "f32", "exp", 2.0, n_targets=3, guard_r=gr, guard_f=gf, train_r=tr,
                         train_f=tf, pfa=pfa, seed=(5, R, F))
    x = synth.generate(spec)
    say("edge", form, case)
    mask, st, th = _run(x, spec.window, form)
    check_full(x, spec.window, mask, st, th, form)


@pytest.mark.parametrize("form", ["plain", "tiled", "direct"])
def test_strided_and_misaligned(form):
    """ld > cols, ld_mask > cols and a map pointer that is not 16-byte
    aligned (vector paths must fall back)."""
    rng = np.random.default_rng(3)
    R, F = 150, 333
    big = torch.from_numpy(rng.exponential(1.0, size=(R, F + 9)).astype(np.float32)).to(DEV)
    win = (2, 3, 7, 11, 1e-3)
    for off in (0, 1, 3):
        xv = big[:, off:off + F]
        mbig = torch.zeros((R, F + 5), dtype=torch.uint8, device=DEV)
        mv = mbig[:, 1:F + 1] if off else mbig[:, :F]
        say("strided", form, off)
        C.cfar2d(xv, win, FORMS[form], mask=mv)
        torch.cuda.synchronize()
        x_np = xv.cpu().numpy()
        check_full(x_np, win, mv.cpu().numpy())
        # columns outside the view are untouched
        assert int(mbig[:, F + 1:].sum().item()) == 0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_sat2d_plain(dtype):
    rng = np.random.default_rng(7)
    for R, F in [(1, 1), (31, 257), (200, 700), (1000, 513)]:
        x = rng.lognormal(0.0, 1.0, size=(R, F)).astype(np.float32 if dtype == "f32" else np.float64)
        say("sat2d plain", dtype, R, F)
        S = C.sat2d(torch.from_numpy(x).to(DEV), C.PLAIN)
        torch.cuda.synchronize()
        ref = oracle.sat(x)[1:, 1:]
        np.testing.assert_allclose(S.cpu().numpy(), ref, rtol=1e-12, atol=0)


def test_sat2d_plain_integer_exact():
    rng = np.random.default_rng(8)
    x = rng.integers(0, 256, size=(777, 1029)).astype(np.float32)
    S = C.sat2d(torch.from_numpy(x).to(DEV), C.PLAIN)
    torch.cuda.synchronize()
    assert np.array_equal(S.cpu().numpy(), oracle.sat(x)[1:, 1:])


def test_sat2d_tiled_layout():
    rng = np.random.default_rng(9)
    for R, F in [(1, 1), (33, 65), (300, 500)]:
        x = rng.lognormal(0.0, 1.0, size=(R, F)).astype(np.float32)
        say("sat2d tiled", R, F)
        buf = C.sat2d(torch.from_numpy(x).to(DEV), C.TILED)
        torch.cuda.synchronize()
        S = decode_tiled_sat(buf.cpu().numpy(), R, F)
        ref = oracle.sat(x)[1:, 1:]
        # FP32 local sums hold at most 32 x 32 cells: error within a few
        # FP32 ulps of the local sum, far below the SAT entries themselves
        np.testing.assert_allclose(S, ref, rtol=1e-6, atol=0)
        # the local region itself: integer maps decode exactly
    xi = rng.integers(0, 64, size=(97, 131)).astype(np.float32)
    buf = C.sat2d(torch.from_numpy(xi).to(DEV), C.TILED)
    torch.cuda.synchronize()
    assert np.array_equal(decode_tiled_sat(buf.cpu().numpy(), 97, 131), oracle.sat(xi)[1:, 1:])


def test_repeat_is_bitwise_deterministic():
    spec = synth.config2(1024, 1024)
    x = torch.from_numpy(synth.generate(spec)).to(DEV)
    outs = []
    for _ in range(3):
        mask = torch.empty(x.shape, dtype=torch.uint8, device=DEV)
        st = torch.empty(x.shape, dtype=torch.float64, device=DEV)
        C.cfar2d(x, spec.window, C.TILED, mask=mask, train_sum=st)
        torch.cuda.synchronize()
        outs.append((mask.cpu().numpy(), st.cpu().numpy()))
    for m, s in outs[1:]:
        assert np.array_equal(m, outs[0][0]) and np.array_equal(s.view(np.int64), outs[0][1].view(np.int64))


def test_plans_give_the_same_answer():
    """Every tile plan computes the same detector (within the parity rule)."""
    spec = synth.config2(700, 900)
    x_np = synth.generate(spec)
    x = torch.from_numpy(x_np).to(DEV)
    ref = oracle.cfar2d(x_np, *spec.window)
    for k in (2, 4, 8):
        for rs in (1, 7, 64, 700):
            mask = torch.empty(x.shape, dtype=torch.uint8, device=DEV)
            st = torch.empty(x.shape, dtype=torch.float64, device=DEV)
            say("plan", k, rs)
            C.cfar2d_with_plan(x, spec.window, k, rs, mask=mask, train_sum=st)
            torch.cuda.synchronize()
            check_full(x_np, spec.window, mask.cpu().numpy(), st.cpu().numpy(), None, "tiled", ref=ref)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_ring_modes_agree(dtype):
    """The interior loop's three row sources (every row from the LDS ring,
    guard rows from the ring, no ring) give the same mask, bit for bit, and
    match the oracle; windows and ring budgets chosen so each mode is taken
    for each k."""
    for (g, t, cols) in [(1, 2, 1100), (2, 5, 1102), (4, 12, 1101), (2, 3, 1024)]:
        # cols % 4 == 0, % 2 only, odd, % 8 == 0: border strips take the EDGE
        # mode or the general one
        spec = synth.MapSpec(600, cols, dtype, "exp", 1.0, n_targets=20, guard_r=g, guard_f=g, train_r=t,
                             train_f=t, pfa=1e-4, seed=(21, g, t))
        x_np = synth.generate(spec)
        x = torch.from_numpy(x_np).to(DEV)
        ref = oracle.cfar2d(x_np, *spec.window)
        for k in (2, 4, 8):
            masks = []
            for ring in (0, 2 * 1024, 8 * 1024, 24 * 1024, 65536):
                mask = torch.empty(x.shape, dtype=torch.uint8, device=DEV)
                say("ring", dtype, g, t, k, ring)
                C.cfar2d_with_plan(x, spec.window, k, 64, mask=mask, ring_bytes=ring)
                torch.cuda.synchronize()
                masks.append(mask.cpu().numpy())
            check_full(x_np, spec.window, masks[0], None, None, "tiled", ref=ref)
            for m in masks[1:]:
                assert np.array_equal(m, masks[0])


@pytest.mark.parametrize("cols", [1101, 1102, 1103, 1100])
def test_padded_rows_and_right_aligned_last_strip(cols):
    """Maps whose rows are 16-byte aligned (padded leading dimension) but whose
    width is not a multiple of k: the last strip is right-aligned, its loads
    and mask stores are not vector-aligned; every plan gives the oracle's
    mask and the padding of the mask rows stays untouched."""
    R, ldx = 300, 1112
    spec = synth.MapSpec(R, cols, "f32", "exp", 1.0, n_targets=10, guard_r=2, guard_f=3, train_r=5, train_f=9,
                         pfa=1e-4, seed=(22, cols))
    x_np = synth.generate(spec)
    big = torch.zeros((R, ldx), dtype=torch.float32, device=DEV)
    big[:, :cols] = torch.from_numpy(x_np).to(DEV)
    xv = big[:, :cols]
    ref = oracle.cfar2d(x_np, *spec.window)
    for k in (2, 4, 8):
        for ring in (0, 12288):
            mbig = torch.full((R, ldx), 7, dtype=torch.uint8, device=DEV)
            mv = mbig[:, :cols]
            say("padded", cols, k, ring)
            C.cfar2d_with_plan(xv, spec.window, k, 64, mask=mv, ring_bytes=ring)
            torch.cuda.synchronize()
            check_full(x_np, spec.window, mv.cpu().numpy(), None, None, "tiled", ref=ref)
            assert (mbig[:, cols:].cpu().numpy() == 7).all()


def test_plain_window_wider_than_strips():
    """PLAIN form with a column half-width above what a 512-column strip
    holds (the per-cell stencil), on one map: every cell against the oracle."""
    spec = synth.MapSpec(37, 1200, "f64", "exp", 2.0, n_targets=2, guard_r=1, guard_f=2, train_r=3,
                         train_f=300, pfa=1e-3, seed=(41,))
    x = synth.generate(spec)
    say("plain wide window", spec.rows, spec.cols, spec.window)
    mask, st, th = _run(x, spec.window, "plain")
    check_full(x, spec.window, mask, st, th, "plain")
