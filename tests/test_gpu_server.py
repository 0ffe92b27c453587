"""The streaming server (cfar_server_create / cfar_submit / cfar_poll /
cfar_server_shutdown / cfar_server_destroy) on the GPU: each frame's result
is the same alone and in the mix, back-pressure, admission by device
memory, and both shutdown modes."""
import ctypes
import time

import numpy as np
import pytest
import torch

from paper_2012_11077_amd import cfar2d as C
from paper_2012_11077_amd import synth
from parity import check_full, say

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _frames(n, seed, rows=(40, 400), cols=(30, 500)):
    specs = synth.config3_specs(n=n, seed=seed, rows=rows, cols=cols)
    return specs, [synth.generate(s) for s in specs]


def _alone(x_np, win):
    x = torch.from_numpy(x_np).to(DEV)
    m = torch.empty(x.shape, dtype=torch.uint8, device=DEV)
    C.cfar2d(x, win, C.TILED, mask=m)
    torch.cuda.synchronize()
    return m.cpu().numpy()


def _drain(srv, tickets, timeout_s=60.0):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < len(tickets):
        assert time.time() < t_end, "server did not complete %d frames" % (len(tickets) - len(got))
        for c in srv.poll(64, 20000):
            got[c.ticket] = c
    return got


def test_alone_equals_in_mix():
    """Host (page-locked) and device frames of many sizes, windows and Pfa,
    submitted together over several HIP streams: every mask equals the one
    the frame gets alone, and matches the oracle."""
    specs, xs = _frames(40, seed=31)
    ref = [_alone(x, s.window) for x, s in zip(xs, specs)]
    with C.Server(device_budget_bytes=256 << 20, max_inflight_frames=16, n_hip_streams=3,
                  queue_depth=64, max_batch_frames=6) as srv:
        keep, tickets = [], {}
        for k, x in enumerate(xs):
            if k % 4 == 0:   # host frame, page-locked by the library
                xh = C.host_empty(x.shape, torch.from_numpy(x).dtype)
                xh.copy_(torch.from_numpy(x))
                mh = C.host_empty(x.shape, torch.uint8)
                mh.fill_(7)
            elif k % 4 == 2:  # host frame, torch pinned memory
                xh = torch.from_numpy(x).pin_memory()
                mh = torch.full(x.shape, 7, dtype=torch.uint8).pin_memory()
            else:            # device frame
                xh = torch.from_numpy(x).to(DEV)
                mh = torch.full(x.shape, 7, dtype=torch.uint8, device=DEV)
            keep.append((xh, mh))
        torch.cuda.synchronize()
        # every frame is ready before the first submit: they arrive together
        # and the server batches them
        for k, (s, (xh, mh)) in enumerate(zip(specs, keep)):
            t = None
            while t is None:
                t = srv.submit(xh, s.window, mh, tag=k)
            tickets[t] = k
        say("server mix", len(tickets))
        got = _drain(srv, tickets)
        st = srv.stats()
    torch.cuda.synchronize()
    for t, c in got.items():
        k = tickets[t]
        assert c.status == C.CFAR_OK and c.user_tag == k
        assert c.t_submit_ns <= c.t_start_ns <= c.t_done_ns
        m = keep[k][1].cpu().numpy()
        assert np.array_equal(m, ref[k]), k
    for k in range(0, len(specs), 7):
        check_full(xs[k], specs[k].window, keep[k][1].cpu().numpy())
    assert st.completed == len(specs) and st.failed == 0
    assert st.batches < len(specs)        # frames were batched together


def test_backpressure_and_small_budget():
    """A tiny queue gives CFAR_EAGAIN; a budget that holds only a few frames
    admits them as memory frees up; every frame still completes."""
    # frames of about 5 MB (input and mask), a budget of 16 MB: at most three
    # on the device at once, each taking its copies' time (about 0.1 ms)
    specs, xs = _frames(30, seed=32, rows=(900, 1100), cols=(900, 1100))
    ref = [_alone(x, s.window) for x, s in zip(xs, specs)]
    budget = 16 << 20
    with C.Server(device_budget_bytes=budget, max_inflight_frames=4, n_hip_streams=2,
                  queue_depth=3, max_batch_frames=2) as srv:
        # every frame is page-locked before the first submit, so the submits
        # come faster than the device completes frames
        keep = [(torch.from_numpy(x).pin_memory(), torch.zeros(x.shape, dtype=torch.uint8).pin_memory())
                for x in xs]
        tickets, eagain = {}, 0
        for k, (s, (xh, mh)) in enumerate(zip(specs, keep)):
            while True:
                t = srv.submit(xh, s.window, mh, tag=k)
                if t is not None:
                    tickets[t] = k
                    break
                eagain += 1
                time.sleep(0.0005)
        got = _drain(srv, tickets)
        st = srv.stats()
    assert eagain > 0
    assert st.device_bytes_peak <= budget
    for t, c in got.items():
        assert c.status == C.CFAR_OK
        assert np.array_equal(keep[tickets[t]][1].numpy(), ref[tickets[t]])


def test_frame_larger_than_budget_is_rejected():
    with C.Server(device_budget_bytes=1 << 20, max_inflight_frames=2, n_hip_streams=1,
                  queue_depth=4, max_batch_frames=1) as srv:
        x = torch.zeros((1024, 1024), dtype=torch.float32)
        m = torch.zeros((1024, 1024), dtype=torch.uint8)
        with pytest.raises(C.CfarError) as e:
            srv.submit(x, (1, 1, 2, 2, 1e-3), m)
        assert e.value.code == C.CFAR_EINVAL


@pytest.mark.parametrize("drain", [True, False])
def test_shutdown(drain):
    """drain: queued frames run; no drain: they complete with
    CFAR_ESHUTDOWN untouched.  Submits after shutdown are refused."""
    specs, xs = _frames(24, seed=33, rows=(300, 600), cols=(300, 600))
    srv = C.Server(device_budget_bytes=64 << 20, max_inflight_frames=2, n_hip_streams=1,
                   queue_depth=64, max_batch_frames=1)
    try:
        keep, tickets = [], {}
        for k, (s, x) in enumerate(zip(specs, xs)):
            xh = torch.from_numpy(x).pin_memory()
            mh = torch.full(x.shape, 9, dtype=torch.uint8).pin_memory()
            keep.append((xh, mh))
            t = srv.submit(xh, s.window, mh, tag=k)
            assert t is not None
            tickets[t] = k
        srv.shutdown(drain=drain)
        # shutdown returns only when nothing is in flight: every ticket's
        # completion is already posted
        got = {c.ticket: c for c in srv.poll(len(tickets) + 8, 0)}
        assert set(got) == set(tickets)
        with pytest.raises(C.CfarError) as e:
            srv.submit(keep[0][0], specs[0].window, keep[0][1])
        assert e.value.code == C.CFAR_ESHUTDOWN
    finally:
        srv.close()
    statuses = [c.status for c in got.values()]
    if drain:
        assert all(s == C.CFAR_OK for s in statuses)
        for t, c in got.items():
            k = tickets[t]
            assert np.array_equal(keep[k][1].numpy(), _alone(xs[k], specs[k].window))
    else:
        assert set(statuses) <= {C.CFAR_OK, C.CFAR_ESHUTDOWN}
        for t, c in got.items():
            k = tickets[t]
            if c.status == C.CFAR_ESHUTDOWN:   # never started: mask untouched
                assert c.t_start_ns == 0
                assert (keep[k][1].numpy() == 9).all()
            else:
                assert np.array_equal(keep[k][1].numpy(), _alone(xs[k], specs[k].window))


def test_packed_masks():
    """Host frames submitted with packed masks (int32 words, some with a
    padded row pitch) next to dense ones: every packed mask unpacks to the
    frame's mask alone, padding words stay untouched; packed masks need host
    frames, enough words per row, and known flags."""
    specs, xs = _frames(12, seed=34, rows=(50, 700), cols=(33, 900))
    ref = [_alone(x, s.window) for x, s in zip(xs, specs)]
    with C.Server(device_budget_bytes=128 << 20, max_inflight_frames=8, n_hip_streams=2,
                  queue_depth=32, max_batch_frames=4) as srv:
        keep, tickets = [], {}
        for k, (s, x) in enumerate(zip(specs, xs)):
            xh = C.host_empty(x.shape, torch.from_numpy(x).dtype)
            xh.copy_(torch.from_numpy(x))
            if k % 3 == 2:      # dense
                mh = C.host_empty(x.shape, torch.uint8)
                mh.fill_(5)
            else:               # packed, row pitch of words + (k % 3) padding words
                words = (x.shape[1] + 31) // 32
                buf = C.host_empty((x.shape[0], words + k % 3), torch.int32)
                buf.fill_(-7)
                mh = buf
            t = None
            while t is None:
                t = srv.submit(xh, s.window, mh, tag=k)
            tickets[t] = k
            keep.append((xh, mh))
        got = _drain(srv, tickets)
        dev = torch.from_numpy(xs[0]).to(DEV)
        bad = torch.zeros((xs[0].shape[0], (xs[0].shape[1] + 31) // 32), dtype=torch.int32, device=DEV)
        with pytest.raises(C.CfarError):          # packed needs a host frame
            srv.submit(dev, specs[0].window, bad)
        short = C.host_empty((xs[0].shape[0], max(1, (xs[0].shape[1] + 31) // 32 - 1)), torch.int32)
        if xs[0].shape[1] > 32:
            with pytest.raises((C.CfarError, ValueError)):
                srv.submit(keep[0][0], specs[0].window, short)
        m = C.make_map(keep[2][0], specs[2].window, keep[2][1])
        tk = ctypes.c_uint64()
        assert C.lib().cfar_submit(srv._h, ctypes.byref(m), 4, 0, ctypes.byref(tk)) == C.CFAR_EINVAL
    for t, c in got.items():
        k = tickets[t]
        assert c.status == C.CFAR_OK
        mh = keep[k][1].numpy()
        if mh.dtype == np.uint8:
            assert np.array_equal(mh, ref[k])
            continue
        F = xs[k].shape[1]
        words = (F + 31) // 32
        bits = np.unpackbits(mh[:, :words].view(np.uint32).view(np.uint8), axis=1, bitorder="little")[:, :F]
        assert np.array_equal(bits, ref[k]), k
        assert (mh[:, words:] == -7).all()


def test_failed_batch_fails_only_its_frames(monkeypatch):
    """A batch whose launch reports failure (forced from the host through
    CFAR2D_SERVER_FAIL_TAG, after its device work ran) completes its frames
    with CFAR_EDEVICE; the other frames, in batches of their own, complete
    normally with the right masks, and the failed batch's memory is given
    back (a second round of the same frames holds the same pool bytes)."""
    monkeypatch.setenv("CFAR2D_SERVER_FAIL_TAG", "5")
    specs, xs = _frames(10, seed=35)
    ref = [_alone(x, s.window) for x, s in zip(xs, specs)]
    with C.Server(device_budget_bytes=64 << 20, max_inflight_frames=4, n_hip_streams=2, queue_depth=32,
                  max_batch_frames=1) as srv:
        keep = []
        for s, x in zip(specs, xs):
            xh = C.host_empty(x.shape, torch.float32)
            xh.copy_(torch.from_numpy(x))
            keep.append((xh, C.host_empty(x.shape, torch.uint8)))
        in_use = []
        for rnd, tag0 in enumerate((0, 100)):   # the second round has no failing tag
            tickets = {}
            for k, (s, (xh, mh)) in enumerate(zip(specs, keep)):
                mh.fill_(7)
                t = srv.submit(xh, s.window, mh, tag=tag0 + k)
                assert t is not None
                tickets[t] = k
            got = _drain(srv, tickets)
            st = srv.stats()
            assert st.inflight_frames == 0 and st.queued_frames == 0
            in_use.append(st.device_bytes_in_use)   # the streams' workspaces, no frame blocks
            for t, c in got.items():
                k = tickets[t]
                if rnd == 0 and k == 5:
                    assert c.status == C.CFAR_EDEVICE
                else:
                    assert c.status == C.CFAR_OK
                    assert np.array_equal(keep[k][1].numpy(), ref[k])
        srv.shutdown(drain=True)
        st = srv.stats()
    assert st.failed == 1 and st.completed == 2 * len(xs)
    assert in_use[0] == in_use[1]   # the failed batch gave its frames' memory back


def test_serving_frame_sizes():
    """One frame from each of the 16 serving streams (256 x 128 up to
    4096 x 1024 FP32, the uneven batch's clutter, targets, windows and Pfa),
    two from the largest, submitted together from page-locked memory:
    every mask equals the frame alone and the oracle's."""
    streams = synth.config4_streams(16, 4)
    frames = [synth.stream_frame_spec(st, 0) for st in streams] + [synth.stream_frame_spec(streams[-1], 1)]
    xs = [synth.generate(sp) for sp in frames]
    ref = [_alone(x, sp.window) for x, sp in zip(xs, frames)]
    with C.Server(device_budget_bytes=1 << 30, max_inflight_frames=32, n_hip_streams=4, queue_depth=64,
                  max_batch_frames=8) as srv:
        keep, tickets = [], {}
        for k, (sp, x) in enumerate(zip(frames, xs)):
            xh = C.host_empty(x.shape, torch.float32)
            xh.copy_(torch.from_numpy(x))
            mh = C.host_empty(x.shape, torch.uint8)
            mh.fill_(7)
            keep.append((xh, mh))
        for k, (sp, (xh, mh)) in enumerate(zip(frames, keep)):
            t = srv.submit(xh, sp.window, mh, tag=k)
            assert t is not None
            tickets[t] = k
        got = _drain(srv, tickets)
    for t, c in got.items():
        k = tickets[t]
        assert c.status == C.CFAR_OK
        m = keep[k][1].numpy()
        assert np.array_equal(m, ref[k]), k
        check_full(xs[k], frames[k].window, m)
