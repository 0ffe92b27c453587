"""Batched CA-CFAR through the C ABI: parity per map, the same result alone
and in any batch, graph replay, and the plain per-map form."""
import numpy as np
import pytest
import torch

from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import check_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _small_batch(n=24, seed=3):
    specs = synth.config3_specs(n=n, seed=seed, rows=(20, 300), cols=(8, 300))
    xs_np = [synth.generate(s) for s in specs]
    return specs, xs_np


def _alloc(xs):
    masks = [torch.empty(x.shape, dtype=torch.uint8, device=DEV) for x in xs]
    sts = [torch.empty(x.shape, dtype=torch.float64, device=DEV) for x in xs]
    return masks, sts


@pytest.mark.parametrize("outputs", [True, False])
@pytest.mark.parametrize("form", ["tiled", "plain"])
@pytest.mark.parametrize("flags", [0, C.BATCH_GRAPH])
def test_batched_parity(form, flags, outputs):
    """Small uneven batch on a side stream (kernel classes fork onto the
    library's own streams and join back), with and without the optional
    training-sum output."""
    specs, xs_np = _small_batch()
    xs = [torch.from_numpy(x).to(DEV) for x in xs_np]
    masks, sts = _alloc(xs)
    say("batched", form, flags, outputs, len(xs))
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        C.cfar2d_batched(xs, [s.window for s in specs], C.TILED if form == "tiled" else C.PLAIN,
                         masks=masks, train_sums=sts if outputs else None, flags=flags, stream=side)
    side.synchronize()
    for k, s in enumerate(specs):
        check_full(xs_np[k], s.window, masks[k].cpu().numpy(), sts[k].cpu().numpy() if outputs else None,
                   None, form)


def test_alone_equals_in_mix_and_order_free():
    specs, xs_np = _small_batch(n=20, seed=5)
    xs = [torch.from_numpy(x).to(DEV) for x in xs_np]
    wins = [s.window for s in specs]
    masks, sts = _alloc(xs)
    C.cfar2d_batched(xs, wins, C.TILED, masks=masks, train_sums=sts)
    torch.cuda.synchronize()
    batch = [(m.cpu().numpy(), s.cpu().numpy()) for m, s in zip(masks, sts)]
    # alone
    for k in range(len(xs)):
        m = torch.empty(xs[k].shape, dtype=torch.uint8, device=DEV)
        s = torch.empty(xs[k].shape, dtype=torch.float64, device=DEV)
        C.cfar2d(xs[k], wins[k], C.TILED, mask=m, train_sum=s)
        torch.cuda.synchronize()
        assert np.array_equal(m.cpu().numpy(), batch[k][0])
        assert np.array_equal(s.cpu().numpy().view(np.int64), batch[k][1].view(np.int64))
    # reversed order, and mixed with other maps
    perm = list(reversed(range(len(xs))))
    extra_specs, extra_np = _small_batch(n=6, seed=9)
    xs2 = [xs[p] for p in perm] + [torch.from_numpy(x).to(DEV) for x in extra_np]
    wins2 = [wins[p] for p in perm] + [s.window for s in extra_specs]
    masks2, sts2 = _alloc(xs2)
    C.cfar2d_batched(xs2, wins2, C.TILED, masks=masks2, train_sums=sts2)
    torch.cuda.synchronize()
    for i, p in enumerate(perm):
        assert np.array_equal(masks2[i].cpu().numpy(), batch[p][0])
        assert np.array_equal(sts2[i].cpu().numpy().view(np.int64), batch[p][1].view(np.int64))


def test_graph_replays_match_eager():
    """Replay the captured batch several times on a side stream with other
    work and synchronisations between replays; every replay equals the eager
    result, also after the inputs change in place."""
    specs, xs_np = _small_batch(n=16, seed=7)
    xs = [torch.from_numpy(x).to(DEV) for x in xs_np]
    wins = [s.window for s in specs]
    eager_masks, eager_sts = _alloc(xs)
    C.cfar2d_batched(xs, wins, C.TILED, masks=eager_masks, train_sums=eager_sts, flags=0)
    torch.cuda.synchronize()
    ref = [(m.cpu().numpy(), s.cpu().numpy()) for m, s in zip(eager_masks, eager_sts)]
    side = torch.cuda.Stream()
    masks, sts = _alloc(xs)
    b = C.Batch(xs, wins, C.TILED, masks=masks, train_sums=sts)
    for rep in range(5):
        for m in masks:
            m.fill_(7)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            b.run(C.BATCH_GRAPH, stream=side)
        side.synchronize()
        junk = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)
        torch.cuda.synchronize()
        del junk
        for k in range(len(xs)):
            assert np.array_equal(masks[k].cpu().numpy(), ref[k][0]), (rep, k)
            assert np.array_equal(sts[k].cpu().numpy(), ref[k][1]), (rep, k)
    # change the data in place: the replay must pick up the new values
    for x in xs:
        x.mul_(2.0)
    with torch.cuda.stream(side):
        b.run(C.BATCH_GRAPH, stream=side)
    side.synchronize()
    for k in range(len(xs)):
        assert np.array_equal(masks[k].cpu().numpy(), ref[k][0])
        np.testing.assert_array_equal(sts[k].cpu().numpy(), 2.0 * ref[k][1])


def test_plain_batch_mixed_stencils():
    """One PLAIN batch whose maps take every stencil path: 256-column strips
    (hf <= 60), 512-column strips (61..247) and the per-cell stencil (wider),
    FP32 and FP64 maps, some with the optional outputs; each map against the
    oracle on every cell."""
    wins = [(1, 1, 4, 4, 1e-3), (2, 30, 3, 40, 1e-4), (1, 3, 2, 280, 1e-3), (3, 2, 9, 58, 1e-5),
            (0, 0, 2, 2, 0.5), (4, 4, 24, 24, 1e-6)]
    shapes = [(70, 300), (33, 1500), (41, 900), (200, 129), (1, 1), (257, 513)]
    specs = []
    for k, ((R, F), w) in enumerate(zip(shapes, wins)):
        specs.append(synth.MapSpec(R, F, "f32" if k % 2 == 0 else "f64", "exp", 2.0, n_targets=2,
                                   guard_r=w[0], guard_f=w[1], train_r=w[2], train_f=w[3], pfa=w[4],
                                   seed=(9, k)))
    xs_np = [synth.generate(s) for s in specs]
    xs = [torch.from_numpy(x).to(DEV) for x in xs_np]
    masks, sts = _alloc(xs)
    outs = [sts[k] if k % 3 == 0 else None for k in range(len(xs))]
    say("plain mixed batch", [(s.rows, s.cols, s.window) for s in specs])
    C.cfar2d_batched(xs, [s.window for s in specs], C.PLAIN, masks=masks, train_sums=outs, flags=0)
    torch.cuda.synchronize()
    for k, s in enumerate(specs):
        check_full(xs_np[k], s.window, masks[k].cpu().numpy(),
                   sts[k].cpu().numpy() if outs[k] is not None else None, None, "plain")


def test_wide_guard_rings_alone_and_in_mix():
    """Maps whose guard ring (2 g_r + 2 rows of the strip) exceeds the default
    LDS budget get a ring of their own size and a launch class of their own:
    FP32 maps with guard 7 and FP64 maps with guard 3 (k = 4), an FP32 map
    with guard 4 and a window wide enough for k = 8, mixed with ordinary
    maps. Every map matches the oracle, alone and in the mix."""
    wide = [synth.MapSpec(180, 700, "f32", "exp", n_targets=12, guard_r=7, guard_f=3, train_r=5, train_f=6,
                          pfa=1e-4, seed=(41, i)) for i in range(2)]
    wide += [synth.MapSpec(150, 640, "f64", "exp_ramp", n_targets=8, guard_r=3, guard_f=2, train_r=9, train_f=7,
                           pfa=1e-5, seed=(42, i)) for i in range(2)]
    # a window too wide for k = 4 (k = 8, 512-column strips) with guard 4
    wide += [synth.MapSpec(200, 700, "f32", "exp", n_targets=6, guard_r=4, guard_f=4, train_r=6, train_f=128,
                           pfa=1e-4, seed=(43, 0))]
    for s in wide:
        k, _, _ = C.plan_for(torch.empty((s.rows, s.cols), device=DEV,
                                         dtype=torch.float32 if s.dtype == "f32" else torch.float64), s.window)
        ring = (2 * s.guard_r + 2) * 64 * k * (4 if s.dtype == "f32" else 8)
        assert k == (8 if s.train_f > 60 else 4) and 12288 < ring <= 20480, (s, k, ring)
    small_specs, small_np = _small_batch(n=8, seed=11)
    specs = wide + list(small_specs)
    xs_np = [synth.generate(s) for s in wide] + small_np
    xs = [torch.from_numpy(x).to(DEV) for x in xs_np]
    wins = [s.window for s in specs]
    masks, sts = _alloc(xs)
    say("wide guard rings", len(wide), "in a batch of", len(xs))
    C.cfar2d_batched(xs, wins, C.TILED, masks=masks, train_sums=sts)
    torch.cuda.synchronize()
    for k in range(len(xs)):
        check_full(xs_np[k], wins[k], masks[k].cpu().numpy(), sts[k].cpu().numpy(), None, "tiled")
    for k in range(len(wide)):
        m = torch.empty(xs[k].shape, dtype=torch.uint8, device=DEV)
        C.cfar2d(xs[k], wins[k], C.TILED, mask=m)
        torch.cuda.synchronize()
        assert np.array_equal(m.cpu().numpy(), masks[k].cpu().numpy())
