"""Full benchmark sizes, every cell against the full FP64 oracle.

Each map goes through the launch the benchmark times: a prepared batch
(``Batch``) replayed from its captured graph on a stream of its own, without
the optional outputs.  The whole mask is compared with the oracle's
(eqs. 1-4, the SAT route) outside the near-threshold margin.  The training
sums come from the same launch with the training-sum output switched on: the
kernel runs the same loop and the same arithmetic, which the equal masks of
the two launches confirm; their largest relative error against the oracle
is the precision figure of the chosen form (bound 1e-6).
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import MARGIN, TILED_REL, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
THREADS = min(16, os.cpu_count() or 1)


def _timed_launch(xs, wins, train_sums=None):
    """The benchmark's launch: Batch + graph replay on a non-null stream."""
    masks = [torch.empty(x.shape, dtype=torch.uint8, device=DEV) for x in xs]
    stream = torch.cuda.Stream()
    b = C.Batch(xs, wins, C.TILED, masks=masks, train_sums=train_sums)
    for _ in range(2):
        b.run(C.BATCH_GRAPH, stream=stream)
    stream.synchronize()
    return masks


def _compare(x_np, window, mask, st=None):
    """Mask against the full oracle outside the margin; box-sum error."""
    m_o, st_o, _, thr_o = oracle.cfar2d(x_np, *window, threads=THREADS, counts=False)
    near = oracle.near_threshold(x_np, thr_o, MARGIN)
    bad = (mask != m_o) & ~near
    out = {"cells": int(mask.size), "near": int(near.sum()), "mismatch": int(bad.sum()),
           "detections": int(m_o.sum())}
    if bad.any():
        out["first_mismatch"] = np.argwhere(bad)[:5].tolist()
    if st is not None:
        with np.errstate(divide="ignore", invalid="ignore"):
            rel = np.where(st_o != 0, np.abs(st - st_o) / np.abs(st_o), np.abs(st - st_o))
        out["max_rel_box_sum_err"] = float(rel.max())
    return out


def _single(spec):
    say("fullsize: generating", spec.rows, spec.cols, spec.dtype)
    x_np = synth.generate(spec)
    x = torch.from_numpy(x_np).to(DEV)
    mask = _timed_launch([x], [spec.window])[0]
    st = torch.empty(x.shape, dtype=torch.float64, device=DEV)
    mask_out = _timed_launch([x], [spec.window], train_sums=[st])[0]
    torch.cuda.synchronize()
    m, m2 = mask.cpu().numpy(), mask_out.cpu().numpy()
    same = bool(np.array_equal(m, m2))
    st_np = st.cpu().numpy()
    del st, mask_out
    say("fullsize: oracle on", x_np.size, "cells,", THREADS, "threads")
    r = _compare(x_np, spec.window, m, st_np)
    r["outputs_launch_same_mask"] = same
    say("fullsize", spec.rows, spec.cols, spec.dtype, r)
    return x, x_np, m, r


def test_precision_map_full_oracle():
    """16384 x 16384 FP32, log-normal clutter (about 60 dB), guard 4, training
    24, Pfa 1e-5: the precision workload, every cell."""
    _, _, _, r = _single(synth.config2())
    assert r["outputs_launch_same_mask"]
    assert r["mismatch"] == 0, r
    assert r["max_rel_box_sum_err"] <= TILED_REL, r


def test_plain_scale_map_full_oracle():
    """8192 x 8192 FP64 on a 0-20 dB range ramp, guard 3, training 16, Pfa
    1e-6: the chosen form on the benchmark's launch and the plain FP64 form,
    each against the oracle on every cell."""
    spec = synth.config1()
    x, x_np, m, r = _single(spec)
    assert r["outputs_launch_same_mask"]
    assert r["mismatch"] == 0, r
    assert r["max_rel_box_sum_err"] <= TILED_REL, r
    plain = C.cfar2d(x, spec.window, C.PLAIN)
    torch.cuda.synchronize()
    rp = _compare(x_np, spec.window, plain.cpu().numpy())
    say("fullsize plain form", rp)
    assert rp["mismatch"] == 0, rp


def test_wide_guard_ring_map_full_oracle():
    """8192 x 8192 FP32 with Table I's widest window (guard 8, background
    12): its guard ring (18 rows of the strip) exceeds the default LDS budget
    and takes a launch class of its own; every cell against the oracle."""
    spec = synth.MapSpec(8192, 8192, "f32", "exp_ramp", n_targets=224, guard_r=8, guard_f=8, train_r=12,
                         train_f=12, pfa=1e-4, seed=(71, 8192))
    x, _, _, r = _single(spec)
    k, _, _ = C.plan_for(x, spec.window)
    assert k == 4 and (2 * spec.guard_r + 2) * 64 * k * 4 > 12288
    assert r["outputs_launch_same_mask"]
    assert r["mismatch"] == 0, r
    assert r["max_rel_box_sum_err"] <= TILED_REL, r


def test_uneven_batch_full_oracle():
    """All 512 maps of the uneven batch in one persistent launch, exactly as
    the benchmark runs it; every cell of every map against the oracle."""
    specs = synth.config3_specs()
    say("full batch: generating", len(specs), "maps")
    arrays = [synth.generate(s) for s in specs]
    xs = [torch.from_numpy(a).to(DEV) for a in arrays]
    masks = _timed_launch(xs, [s.window for s in specs])
    torch.cuda.synchronize()
    tot = {"maps": len(specs), "cells": 0, "near": 0, "mismatch": 0, "detections": 0}
    for k, s in enumerate(specs):
        r = _compare(arrays[k], s.window, masks[k].cpu().numpy())
        for key in ("cells", "near", "mismatch", "detections"):
            tot[key] += r[key]
        if r["mismatch"]:
            say("full batch: map", k, s.rows, s.cols, s.window, r)
    say("full batch", tot)
    assert tot["mismatch"] == 0, tot


def test_false_alarm_rate_at_scale():
    """Exponential noise only, 8192 x 8192: the detection rate matches Pfa
    (CA-CFAR's constant false-alarm property)."""
    spec = synth.MapSpec(8192, 8192, "f32", "exp", 3.0, n_targets=0, guard_r=2, guard_f=2,
                         train_r=8, train_f=8, pfa=1e-3, seed=(77,))
    x = torch.from_numpy(synth.generate(spec)).to(DEV)
    mask = C.cfar2d(x, spec.window, C.TILED)
    torch.cuda.synchronize()
    rate = mask.double().mean().item()
    say("FA rate", rate)
    assert abs(rate - 1e-3) < 0.05e-3
