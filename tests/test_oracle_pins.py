"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test names the passage of arXiv 2012.11077 it checks and the independent
source of truth: hand-worked fixtures, numpy/scipy library routines, brute
force direct summation with math.fsum, closed forms of eq. (2), and invariants
of CA-CFAR.  A plausible mistake in the oracle (a dropped corner, a wrong sign
in eq. 2, an off-by-one clip, a transposed axis) fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.signal import convolve2d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Hand-worked fixtures (eqs. 1-4)
# --------------------------------------------------------------------------

def test_golden_ramp_3x3(oracle_mod):
    g = _golden("ramp_3x3.json")
    x = np.array(g["map"], dtype=np.float64)
    assert np.array_equal(oracle_mod.sat(x), np.array(g["expected_sat_padded"], dtype=np.float64))
    mask, st, nt, thr = oracle_mod.cfar2d(x, g["guard_r"], g["guard_f"], g["train_r"], g["train_f"],
                                          g["pfa"])
    assert np.array_equal(st, np.array(g["expected_train_sum"], dtype=np.float64))
    assert np.array_equal(nt, np.array(g["expected_n_train"]))
    assert np.array_equal(mask, np.array(g["expected_mask"], dtype=np.uint8))


def test_golden_spike_5x5(oracle_mod):
    g = _golden("spike_5x5.json")
    x = np.array(g["map"], dtype=np.float64)
    mask, st, nt, thr = oracle_mod.cfar2d(x, g["guard_r"], g["guard_f"], g["train_r"], g["train_f"],
                                          g["pfa"])
    assert np.array_equal(st, np.array(g["expected_train_sum"], dtype=np.float64))
    assert np.array_equal(nt, np.array(g["expected_n_train"]))
    assert np.array_equal(mask, np.array(g["expected_mask"], dtype=np.uint8))
    assert oracle_mod.alpha(8, g["pfa"]) == pytest.approx(g["expected_alpha_n8"], rel=1e-15)
    assert thr[2, 2] == pytest.approx(8.0, rel=1e-15)


# --------------------------------------------------------------------------
# eq. (3): the integral image equals the double cumulative sum
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (13, 17), (64, 33)])
def test_sat_is_double_cumsum_integer_exact(oracle_mod, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.integers(0, 1000, size=shape).astype(np.float64)
    S = oracle_mod.sat(x)
    assert np.all(S[0, :] == 0) and np.all(S[:, 0] == 0)
    ref = np.cumsum(np.cumsum(x, axis=0), axis=1)
    assert np.array_equal(S[1:, 1:], ref)


def test_sat_float_close_to_cumsum(oracle_mod):
    rng = np.random.default_rng(5)
    x = rng.lognormal(0.0, 2.0, size=(200, 150))
    S = oracle_mod.sat(x)
    ref = np.cumsum(np.cumsum(x, axis=0), axis=1)
    np.testing.assert_allclose(S[1:, 1:], ref, rtol=1e-13, atol=0)


# --------------------------------------------------------------------------
# eq. (4) + border clipping: brute force on every tiny map and window
# --------------------------------------------------------------------------

def _brute(x, gr, gf, tr, tf):
    """Training sum (math.fsum) and count by walking the clipped windows."""
    R, F = x.shape
    hr, hf = gr + tr, gf + tf
    st = np.zeros((R, F))
    nt = np.zeros((R, F), dtype=np.int64)
    for i in range(R):
        for j in range(F):
            vals = []
            for a in range(max(0, i - hr), min(R - 1, i + hr) + 1):
                for b in range(max(0, j - hf), min(F - 1, j + hf) + 1):
                    if abs(a - i) <= gr and abs(b - j) <= gf:
                        continue
                    vals.append(x[a, b])
            st[i, j] = math.fsum(vals)
            nt[i, j] = len(vals)
    return st, nt


@pytest.mark.parametrize("R,F", [(1, 1), (1, 5), (4, 1), (3, 7), (7, 7), (6, 5)])
def test_bruteforce_all_windows(oracle_mod, R, F):
    rng = np.random.default_rng(R * 100 + F)
    x = rng.integers(0, 50, size=(R, F)).astype(np.float64)   # integer: every sum exact
    for gr, gf, tr, tf in itertools.product(range(0, 3), range(0, 3), range(0, 3), range(0, 3)):
        if tr + tf == 0:
            continue
        mask, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 1e-2)
        bst, bnt = _brute(x, gr, gf, tr, tf)
        assert np.array_equal(nt, bnt), (gr, gf, tr, tf)
        assert np.array_equal(st, bst), (gr, gf, tr, tf)


def test_bruteforce_float_windows_wider_than_map(oracle_mod):
    rng = np.random.default_rng(11)
    x = rng.lognormal(0.0, 2.0, size=(5, 6))
    for gr, gf, tr, tf in [(0, 0, 4, 4), (1, 2, 3, 1), (4, 4, 4, 4), (0, 3, 0, 2)]:
        mask, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 1e-3)
        bst, bnt = _brute(x, gr, gf, tr, tf)
        assert np.array_equal(nt, bnt)
        np.testing.assert_allclose(st, bst, rtol=1e-13, atol=1e-13 * np.abs(x).sum())


def test_convolution_cross_check(oracle_mod):
    """Clipped window sums equal zero-filled 2D box convolutions ('same' mode):
    zero fill adds nothing, and the same convolution of ones counts cells."""
    rng = np.random.default_rng(3)
    x = rng.integers(0, 100, size=(40, 31)).astype(np.float64)
    gr, gf, tr, tf = 2, 1, 5, 3
    hr, hf = gr + tr, gf + tf
    outer = convolve2d(x, np.ones((2 * hr + 1, 2 * hf + 1)), mode="same")
    inner = convolve2d(x, np.ones((2 * gr + 1, 2 * gf + 1)), mode="same")
    ones = np.ones_like(x)
    n_outer = convolve2d(ones, np.ones((2 * hr + 1, 2 * hf + 1)), mode="same")
    n_inner = convolve2d(ones, np.ones((2 * gr + 1, 2 * gf + 1)), mode="same")
    mask, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 1e-4)
    assert np.array_equal(st, outer - inner)
    assert np.array_equal(nt, (n_outer - n_inner).astype(np.int64))


def test_fsum_error_of_oracle_on_heavy_tailed_map(oracle_mod):
    """The oracle's own FP64 rounding on a log-normal (sigma 2) map stays far
    below the 1e-6 parity bound (checked against math.fsum on sampled cells)."""
    rng = np.random.default_rng(21)
    x = np.exp(2.0 * rng.standard_normal((300, 260)))
    gr, gf, tr, tf = 4, 4, 24, 24
    mask, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 1e-5)
    cells = rng.integers(0, [300, 260], size=(60, 2))
    hr, hf = gr + tr, gf + tf
    for i, j in cells:
        blk = x[max(0, i - hr):i + hr + 1, max(0, j - hf):j + hf + 1]
        gb = x[max(0, i - gr):i + gr + 1, max(0, j - gf):j + gf + 1]
        ref = math.fsum(blk.ravel()) - math.fsum(gb.ravel())
        assert abs(st[i, j] - ref) <= 1e-12 * ref


def test_direct_route_matches_sat_route(oracle_mod):
    """Direct CA-CFAR (Table I, no integral image) on listed cells equals the
    integral-image route on the same cells."""
    rng = np.random.default_rng(8)
    x = rng.integers(0, 30, size=(50, 70)).astype(np.float64)
    gr, gf, tr, tf, pfa = 1, 3, 6, 2, 1e-3
    mask, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, pfa)
    rows = rng.integers(0, 50, size=400)
    cols = rng.integers(0, 70, size=400)
    m2, st2, nt2, thr2 = oracle_mod.cfar2d_cells(x, gr, gf, tr, tf, pfa, rows, cols)
    assert np.array_equal(st2, st[rows, cols])
    assert np.array_equal(nt2, nt[rows, cols])
    assert np.array_equal(thr2, thr[rows, cols])
    assert np.array_equal(m2, mask[rows, cols])


def test_threads_do_not_change_the_oracle(oracle_mod):
    """The per-cell loop split over threads gives bit-identical outputs (the
    all-core timing and the full-size checks rely on it); counts=False only
    drops the training counts."""
    rng = np.random.default_rng(9)
    x = rng.lognormal(0.0, 2.0, size=(301, 257))
    one = oracle_mod.cfar2d(x, 2, 3, 9, 7, 1e-4)
    many = oracle_mod.cfar2d(x, 2, 3, 9, 7, 1e-4, threads=4, counts=False)
    assert many[2] is None
    for a, b in ((one[0], many[0]), (one[1], many[1]), (one[3], many[3])):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


# --------------------------------------------------------------------------
# eq. (2): the scale factor, closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 8, 112, 416, 1472, 3168])
@pytest.mark.parametrize("pfa", [0.5, 1e-1, 1e-3, 1e-4, 1e-6])
def test_alpha_inverts_false_alarm_law(oracle_mod, n, pfa):
    """For square-law noise the false-alarm probability of T = alpha * A is
    (1 + alpha/N)^(-N); the oracle's alpha must give back Pfa."""
    a = oracle_mod.alpha(n, pfa)
    assert a > 0
    back = math.exp(-n * math.log1p(a / n))
    assert back == pytest.approx(pfa, rel=1e-12)


def test_alpha_exact_small_cases(oracle_mod):
    assert oracle_mod.alpha(1, 0.5) == pytest.approx(1.0, rel=1e-15)      # 1/Pfa - 1
    assert oracle_mod.alpha(1, 0.25) == pytest.approx(3.0, rel=1e-15)
    assert oracle_mod.alpha(2, 0.25) == pytest.approx(2.0, rel=1e-15)     # 2(Pfa^-1/2 - 1)
    assert oracle_mod.alpha(2, 1.0 / 9.0) == pytest.approx(4.0, rel=1e-14)
    assert oracle_mod.alpha(8, 2.0 ** -8) == pytest.approx(8.0, rel=1e-15)


def test_alpha_limit_and_monotone(oracle_mod):
    pfa = 1e-4
    vals = [oracle_mod.alpha(n, pfa) for n in (1, 4, 16, 64, 256, 1024, 10 ** 6)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert vals[-1] == pytest.approx(-math.log(pfa), rel=1e-5)


def test_printed_sign_of_eq2_is_rejected(oracle_mod):
    """eq. (2) as printed, N (Pfa^(1/N) - 1), is negative for 0 < Pfa < 1, so
    T < 0 and every positive cell would be a detection.  The oracle's factor
    is positive and the constant-map test below fails for the printed sign."""
    for n in (8, 416):
        printed = n * (1e-4 ** (1.0 / n) - 1.0)
        assert printed < 0
        assert oracle_mod.alpha(n, 1e-4) > 0


# --------------------------------------------------------------------------
# Closed forms on constant maps (eqs. 1, 2, border clipping)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("c", [1.0, 7.0, 1024.0])
def test_constant_map_closed_form(oracle_mod, c):
    x = np.full((23, 19), c)
    gr, gf, tr, tf = 2, 1, 4, 6
    m_hi, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 0.6)
    assert np.array_equal(st, c * nt.astype(np.float64))         # A = c exactly
    assert np.all(nt > 0)
    assert np.all(m_hi == 1)        # alpha < 1 for every N at Pfa = 0.6
    for pfa in (0.3, 1e-2, 1e-6):
        m_lo, _, _, _ = oracle_mod.cfar2d(x, gr, gf, tr, tf, pfa)
        assert np.all(m_lo == 0)    # alpha > 1 for every N at Pfa <= 0.3


def test_no_training_cells_means_no_detection(oracle_mod):
    x = np.array([[5.0]])
    m, st, nt, thr = oracle_mod.cfar2d(x, 0, 0, 3, 3, 0.5)
    assert nt[0, 0] == 0 and m[0, 0] == 0 and np.isinf(thr[0, 0])
    # guard covers the whole (clipped) window: N = 0 everywhere
    x = np.ones((3, 4))
    m, st, nt, thr = oracle_mod.cfar2d(x, 3, 4, 1, 1, 0.5)
    assert np.all(nt == 0) and np.all(m == 0)


def test_equality_is_not_a_detection(oracle_mod):
    """eq. (1) declares H1 only for CUT > T.  With N = 1 and Pfa = 0.5,
    alpha = 1, so T equals the single training cell."""
    x = np.array([[3.0, 3.0]])
    m, st, nt, thr = oracle_mod.cfar2d(x, 0, 0, 0, 1, 0.5)
    assert np.array_equal(nt, [[1, 1]])
    assert np.array_equal(thr, [[3.0, 3.0]])
    assert np.array_equal(m, [[0, 0]])


# --------------------------------------------------------------------------
# Invariants of CA-CFAR
# --------------------------------------------------------------------------

def test_power_of_two_scale_invariance(oracle_mod):
    rng = np.random.default_rng(4)
    x = rng.exponential(1.0, size=(80, 60))
    x[40, 30] += 60.0
    m, st, nt, thr = oracle_mod.cfar2d(x, 2, 2, 6, 5, 1e-3)
    for k in (-7, 3, 20):
        m2, st2, nt2, thr2 = oracle_mod.cfar2d(x * 2.0 ** k, 2, 2, 6, 5, 1e-3)
        assert np.array_equal(m2, m)
        assert np.array_equal(st2, st * 2.0 ** k)


def test_flip_and_transpose_symmetry(oracle_mod):
    rng = np.random.default_rng(6)
    x = rng.integers(0, 40, size=(30, 41)).astype(np.float64)
    gr, gf, tr, tf = 1, 2, 3, 5
    m, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 1e-2)
    for flip in (np.flipud, np.fliplr):
        m2, st2, nt2, _ = oracle_mod.cfar2d(flip(x), gr, gf, tr, tf, 1e-2)
        assert np.array_equal(st2, flip(st))
        assert np.array_equal(nt2, flip(nt))
        assert np.array_equal(m2, flip(m))
    m3, st3, nt3, _ = oracle_mod.cfar2d(np.ascontiguousarray(x.T), gf, gr, tf, tr, 1e-2)
    assert np.array_equal(st3, st.T) and np.array_equal(m3, m.T)


def test_crop_consistency(oracle_mod):
    """Cells at least one outer half-width inside a crop see the same window."""
    rng = np.random.default_rng(7)
    x = rng.integers(0, 40, size=(60, 70)).astype(np.float64)
    gr, gf, tr, tf = 1, 1, 4, 3
    hr, hf = gr + tr, gf + tf
    m, st, nt, thr = oracle_mod.cfar2d(x, gr, gf, tr, tf, 1e-3)
    r0, c0 = 11, 17
    xc = x[r0:r0 + 30, c0:c0 + 25]
    mc, stc, ntc, _ = oracle_mod.cfar2d(xc, gr, gf, tr, tf, 1e-3)
    inner = (slice(hr, 30 - hr), slice(hf, 25 - hf))
    full = (slice(r0 + hr, r0 + 30 - hr), slice(c0 + hf, c0 + 25 - hf))
    assert np.array_equal(stc[inner], st[full])
    assert np.array_equal(mc[inner], m[full])


def test_false_alarm_rate_on_exponential_noise(oracle_mod):
    """With i.i.d. exponential (square-law) noise, CA-CFAR with the eq. (2)
    factor holds the false-alarm rate at Pfa, including at clipped border
    cells where N is smaller.  Spread is taken across maps, since overlapping
    windows correlate neighbouring cells."""
    n_maps, R, F = 24, 256, 256
    gr, gf, tr, tf = 2, 2, 8, 8
    hr, hf = gr + tr, gf + tf
    border = np.ones((R, F), dtype=bool)
    border[hr:R - hr, hf:F - hf] = False
    for pfa in (1e-1, 1e-2):
        rates, brates = [], []
        for k in range(n_maps):
            x = np.random.default_rng((31, k)).standard_exponential((R, F))
            m, _, _, _ = oracle_mod.cfar2d(x, gr, gf, tr, tf, pfa)
            rates.append(m.mean())
            brates.append(m[border].mean())
        for r in (np.array(rates), np.array(brates)):
            sd = r.std(ddof=1) / math.sqrt(n_maps)
            assert abs(r.mean() - pfa) <= 5 * sd + 1e-12, (pfa, r.mean(), sd)
            assert abs(r.mean() - pfa) <= 0.1 * pfa


# ---------------------------------------------------------------------------
# Detection lists and packed masks (the H1 cells of eq. 1, handed on)
# ---------------------------------------------------------------------------
def test_detection_list_order_and_content(oracle_mod):
    rng = np.random.default_rng(5)
    m = (rng.random((7, 13)) < 0.2).astype(np.uint8)
    x = rng.random((7, 13))
    t = rng.random((7, 13))
    recs = oracle_mod.detection_list(m, x, t)
    # row-major order is the lexicographic order of (row, col); one record per set cell
    idx = [(r[0], r[1]) for r in recs]
    assert idx == sorted(idx) and len(set(idx)) == len(idx) == int(m.sum())
    assert idx == [tuple(v) for v in np.argwhere(m != 0).tolist()]
    for (i, j, c, th) in recs:
        assert c == x[i, j] and th == t[i, j]
    assert all(np.isnan(r[3]) for r in oracle_mod.detection_list(m, x))
    assert oracle_mod.detection_list(np.zeros((3, 4), np.uint8), x[:3, :4]) == []


def test_pack_mask_round_trip(oracle_mod):
    rng = np.random.default_rng(6)
    for F in (1, 31, 32, 33, 100):
        m = (rng.random((5, F)) < 0.5).astype(np.uint8)
        p = oracle_mod.pack_mask(m)
        assert p.shape == (5, (F + 31) // 32)
        bits = np.unpackbits(p.view(np.uint8), axis=1, bitorder="little")[:, :F]
        assert np.array_equal(bits, m)
        assert int(sum(bin(int(v)).count("1") for v in p.ravel())) == int(m.sum())
