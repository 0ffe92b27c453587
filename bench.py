#!/usr/bin/env python3
"""Benchmark of integral-image 2D CA-CFAR on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]

A step is one pass of the whole hot path over one batch of synthetic input:
threshold tables, then the fused tiled CA-CFAR (tile-local prefix sums with
FP64 carries, eight corners, threshold, decision) over every map, as one
persistent launch replayed from a captured hipGraph.  Inputs are resident in
device memory before the timed region starts.

Default workload: the uneven batch of 512 FP32 maps (rows U[200, 4096] x
cols U[64, 2048], per-map window and Pfa).  Beside it the same maps go
through the plain per-map FP64 form (FP64 integral image in device memory,
then the eight-corner stencil, one map after the other) and the CPU oracle
is timed on a bounded sample of the maps.

Prints ONE JSON line.  ``value`` is cells/s of the chosen (tiled) form;
``roofline`` prices the dominant kernel (the persistent CA-CFAR kernel) at
its algorithmic bytes (map read once + mask written once) against HBM peak.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "CA-CFAR cells/s & % HBM peak, chosen vs plain form at equal mask; p99 latency"
# rocprofv3 counter summaries of the fused kernel, per workload
TRAFFIC_FILES = {"batched": os.path.join(ROOT, "profiles", "fused_kernel_uneven_batch_traffic.json"),
                 "precision": os.path.join(ROOT, "profiles", "fused_kernel_16k_f32_map_traffic.json"),
                 "plain_scale": os.path.join(ROOT, "profiles", "fused_kernel_8k_f64_map_traffic.json")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Hash of the sources that decide the fused kernel's memory traffic: the
    kernel, its descriptor layout and the host planner."""
    h = hashlib.sha256()
    for name in ("fused.hip", "internal.h", "cfar2d_host.cpp"):
        with open(os.path.join(ROOT, "paper_2012_11077_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter runs of the workload, if they were taken on the current kernel
    source."""
    if workload not in TRAFFIC_FILES:
        return None
    try:
        with open(TRAFFIC_FILES[workload]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_source_sha():
        return None
    return t


def _counter_per_dispatch(path, counter, kernel_substr, reduce="mean"):
    """A rocprofv3 counter over the dispatches of the kernels whose name
    contains kernel_substr (sqlite database(s) under path): reduce "max" =
    the largest dispatch, "mean" = the mean per launch group, where a group
    holds one dispatch of each distinct kernel (the kernel classes of one
    batched launch run concurrently).  Returns (value, dispatches)."""
    import glob
    import sqlite3
    vals, names = {}, set()
    for db in glob.glob(os.path.join(path, "**", "*.db"), recursive=True):
        c = sqlite3.connect(db)
        for name, disp, v in c.execute("select kernel_name, dispatch_id, value from counters_collection "
                                       "where counter_name = ?", (counter,)):
            if kernel_substr in name:
                vals[(db, disp)] = vals.get((db, disp), 0.0) + float(v)
                names.add(name)
        c.close()
    if not vals:
        raise SystemExit("no %s samples for %r under %s" % (counter, kernel_substr, path))
    if reduce == "max":
        return max(vals.values()), len(vals)
    groups = len(vals) / max(1, len(names))
    return sum(vals.values()) / groups, len(vals)


def record_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, command):
    """HBM bytes per launch of the fused kernel from two rocprofv3 counter runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
    same counter reads for the 1 GiB device copy of --copy-probe; written to
    the traffic file with the kernel source hash."""
    copy_bytes = float(1 << 30)
    # the probe's copies are its largest dispatches (the fill before them reads nothing)
    cf, _ = _counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE", "", reduce="max")
    cw, _ = _counter_per_dispatch(copy_write_dir, "WRITE_SIZE", "", reduce="max")
    f_scale, w_scale = copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)
    fk, n1 = _counter_per_dispatch(fetch_dir, "FETCH_SIZE", "fused_kernel")
    wk, n2 = _counter_per_dispatch(write_dir, "WRITE_SIZE", "fused_kernel")
    t = {"kernel": "fused_kernel", "workload": workload, "kernel_sha": kernel_source_sha(),
         "fetch_kib_per_launch": round(fk, 1), "write_kib_per_launch": round(wk, 1),
         "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
         "bytes_per_launch": int(fk * 1024.0 * f_scale + wk * 1024.0 * w_scale),
         "dispatches": [n1, n2], "command": command}
    with open(TRAFFIC_FILES[workload], "w") as f:
        json.dump(t, f, indent=1)
    print(json.dumps(t), flush=True)


def percentile(v, q):
    v = sorted(v)
    if not v:
        return None
    k = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def oracle_threads():
    """Host threads the all-core oracle run uses: OMP_NUM_THREADS if set (the
    host's share), else every core."""
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return max(1, os.cpu_count() or 1)


def cpu_baseline(specs, arrays, gpu_masks=None, reps=3):
    """The FP64 oracle as it stands over the whole workload: one pass on one
    thread, then the per-cell loop on all host threads (median of reps).
    The all-thread run's masks are compared with the GPU's outside the
    near-threshold margin (mismatches expected: none)."""
    import oracle
    oracle.build(force=False)
    cells = sum(s.cells for s in specs)
    t0 = time.perf_counter()
    for s, x in zip(specs, arrays):
        oracle.cfar2d(x, *s.window, threads=1, counts=False)
    t_one = time.perf_counter() - t0
    nt = oracle_threads()
    times, mismatch, near = [], 0, 0
    for rep in range(reps):
        t = 0.0
        for k, (s, x) in enumerate(zip(specs, arrays)):
            t0 = time.perf_counter()
            m_o, _, _, thr_o = oracle.cfar2d(x, *s.window, threads=nt, counts=False)
            t += time.perf_counter() - t0
            if rep == 0 and gpu_masks is not None:
                nr = oracle.near_threshold(x, thr_o)
                mismatch += int(((gpu_masks[k] != m_o) & ~nr).sum())
                near += int(nr.sum())
        times.append(t)
    t_all = float(np.median(times))
    return {"value": cells / t_all, "unit": "cells/s", "cores": nt, "kind": "oracle",
            "single_thread_cells_per_s": cells / t_one, "single_thread_s": round(t_one, 2),
            "all_threads_s": round(t_all, 3), "all_threads_reps": reps,
            "sample": "every map of the workload (%d maps, %d cells): FP64 oracle once on 1 thread, then its "
                      "per-cell loop on %d threads, median of %d" % (len(specs), cells, nt, reps),
            "gpu_vs_oracle": ({"mask_cells_differing_outside_margin": mismatch, "near_threshold_cells": near,
                               "margin": "|X - T| <= 1e-5 |T|"} if gpu_masks is not None else None)}


def precision_report():
    """The precision workload (16384 x 16384 FP32, log-normal clutter, guard
    4, training 24, Pfa 1e-5) on the benchmark's launch of the chosen form,
    with and without the training-sum output, and on the plain FP64 form:
    largest relative box-sum error against the FP64 oracle, near-threshold
    cells, mask cells differing outside the margin."""
    import torch
    import oracle
    from paper_2012_11077_amd import cfar2d as C
    from paper_2012_11077_amd import synth
    dev = torch.device("cuda:0")
    spec = synth.config2()
    x_np = synth.generate(spec)
    x = torch.from_numpy(x_np).to(dev)
    stream = torch.cuda.Stream()
    out = {}
    masks = {}
    for name, form, with_st in (("chosen", C.TILED, False), ("chosen_with_sums", C.TILED, True),
                                ("plain", C.PLAIN, True)):
        mask = torch.empty(x.shape, dtype=torch.uint8, device=dev)
        st = torch.empty(x.shape, dtype=torch.float64, device=dev) if with_st else None
        b = C.Batch([x], [spec.window], form, masks=[mask], train_sums=[st] if st is not None else None)
        for _ in range(2):
            b.run(C.BATCH_GRAPH, stream=stream)
        stream.synchronize()
        masks[name] = mask.cpu().numpy()
        out[name] = {"st": st.cpu().numpy() if st is not None else None}
        del b, st
    torch.cuda.synchronize()
    m_o, st_o, _, thr_o = oracle.cfar2d(x_np, *spec.window, threads=oracle_threads(), counts=False)
    near = oracle.near_threshold(x_np, thr_o)
    rep = {"workload": "16384x16384 FP32, log-normal clutter sigma 2, 1000 targets 8-30 dB, guard 4x4, "
                       "training 24x24, Pfa 1e-5, seed 2",
           "near_threshold_cells": int(near.sum()), "oracle_detections": int(m_o.sum()),
           "chosen_masks_equal_with_and_without_sums": bool(np.array_equal(masks["chosen"],
                                                                           masks["chosen_with_sums"]))}
    for name in ("chosen", "plain"):
        rep[name + "_mask_cells_differing_outside_margin"] = int(((masks[name] != m_o) & ~near).sum())
    with np.errstate(divide="ignore", invalid="ignore"):
        for name, key in (("chosen_with_sums", "chosen"), ("plain", "plain")):
            st = out[name]["st"]
            rel = np.where(st_o != 0, np.abs(st - st_o) / np.abs(st_o), 0.0)
            rep[key + "_max_rel_box_sum_err"] = float(rel.max())
    # the FP32-tile-local integral image with FP64 carries (sat2d's TILED
    # layout): training sums from its corners, against the oracle's
    buf = C.sat2d(x, C.TILED).cpu().numpy()
    torch.cuda.synchronize()
    rep["fp32_local_sat_max_rel_box_sum_err"] = fp32_local_box_err(buf, spec.rows, spec.cols, spec.window, st_o)
    return rep


def fp32_local_box_err(buf, rows, cols, window, st_o, block=1024):
    """Largest relative error of the training sums (eq. 4, clipped windows)
    taken from the corners of sat2d's TILED layout (FP32 sums inside 32 x 32
    tiles, FP64 row and column lines every 32 rows / columns; decoded in FP64
    here) against the oracle's training sums st_o."""
    line = 32

    def up(v):
        return (v + 255) // 256 * 256

    raw = np.ascontiguousarray(buf).view(np.uint8)
    n_i, n_j = (rows + line - 1) // line, (cols + line - 1) // line
    loc_b, row_b = up(rows * cols * 4), up(n_i * cols * 8)
    loc = raw[:rows * cols * 4].view(np.float32).reshape(rows, cols)
    rowline = raw[loc_b:loc_b + n_i * cols * 8].view(np.float64).reshape(n_i, cols)
    colline = raw[loc_b + row_b:loc_b + row_b + n_j * rows * 8].view(np.float64).reshape(n_j, rows)
    tj = np.arange(cols) // line
    cj = np.maximum(tj * line - 1, 0)
    # S with a zero row and column in front: P[i+1, j+1] = S(i, j)
    P = np.zeros((rows + 1, cols + 1))
    for i0 in range(0, rows, block):
        i1 = min(i0 + block, rows)
        ti = np.arange(i0, i1) // line
        P[i0 + 1:i1 + 1, 1:] = (rowline[ti, :] + colline[tj, i0:i1].T - rowline[ti][:, cj] * (tj > 0)[None, :]
                                + loc[i0:i1].astype(np.float64))
    gr, gf, tr, tf, _ = window
    hr, hf = gr + tr, gf + tf
    jj = np.arange(cols)
    co0, co1 = np.maximum(jj - hf, 0), np.minimum(jj + hf, cols - 1) + 1
    ci0, ci1 = np.maximum(jj - gf, 0), np.minimum(jj + gf, cols - 1) + 1
    worst = 0.0
    for i0 in range(0, rows, block):
        ii = np.arange(i0, min(i0 + block, rows))
        ro0, ro1 = np.maximum(ii - hr, 0), np.minimum(ii + hr, rows - 1) + 1
        ri0, ri1 = np.maximum(ii - gr, 0), np.minimum(ii + gr, rows - 1) + 1
        outer = P[ro1][:, co1] - P[ro0][:, co1] - P[ro1][:, co0] + P[ro0][:, co0]
        inner = P[ri1][:, ci1] - P[ri0][:, ci1] - P[ri1][:, ci0] + P[ri0][:, ci0]
        ref = st_o[ii]
        with np.errstate(divide="ignore", invalid="ignore"):
            rel = np.where(ref != 0, np.abs((outer - inner) - ref) / np.abs(ref), 0.0)
        worst = max(worst, float(rel.max()))
    return worst


# Table I of the paper (workstation, Intel Core i5-6200U): CA-CFAR without and
# with the integral image, seconds, per (guard, background) cells per side
PAPER_TABLE1_S = {(4, 8): (0.126, 0.026), (4, 12): (0.201, 0.016), (8, 8): (0.175, 0.015), (8, 12): (0.184, 0.019)}


def table1_bench(steps=5, warmup=2):
    """Table I on the GPU: the DIRECT form (every cell sums its own training
    cells) against the TILED and PLAIN integral-image forms, at each (guard,
    background) setting, on a map of the paper's record size (1024 range
    bins x 600 slow-time frequency bins, FP64) and on a 16384 x 16384 FP32
    map.  Kernel-sequence time per map with HIP events on one stream."""
    import torch
    from paper_2012_11077_amd import cfar2d as C
    from paper_2012_11077_amd import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    rows = []
    for name, R, F, dt in [("1024x600 FP64 (paper-sized record)", 1024, 600, "f64"),
                           ("16384x16384 FP32", 16384, 16384, "f32")]:
        spec0 = synth.MapSpec(R, F, dt, "exp_ramp", n_targets=max(1, R * F // 300000), guard_r=4, guard_f=4,
                              train_r=8, train_f=8, pfa=1e-4, seed=(71, R))
        x = torch.from_numpy(synth.generate(spec0)).to(dev)
        mask = torch.empty(x.shape, dtype=torch.uint8, device=dev)
        masks = {}
        for (g, b) in PAPER_TABLE1_S:
            win = (g, g, b, b, 1e-4)
            ms = {}
            for fname, form in (("direct", C.DIRECT), ("tiled", C.TILED), ("plain", C.PLAIN)):
                m = C.make_map(x, win, mask)
                ws = torch.empty(C.workspace_bytes([m], form), dtype=torch.uint8, device=dev)
                for _ in range(warmup):
                    C.cfar2d(x, win, form, mask=mask, ws=ws, stream=stream)
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
                ev[0].record(stream)
                for k in range(steps):
                    C.cfar2d(x, win, form, mask=mask, ws=ws, stream=stream)
                    ev[k + 1].record(stream)
                torch.cuda.synchronize()
                ms[fname] = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]))
                masks[fname] = mask.clone()
                del ws
            same = int((masks["direct"] != masks["tiled"]).sum().item())
            row = {"map": name, "guard": g, "background": b, "window": [2 * (g + b) + 1] * 2,
                   "direct_ms": round(ms["direct"], 4), "tiled_ms": round(ms["tiled"], 4),
                   "plain_ms": round(ms["plain"], 4),
                   "direct_over_tiled": round(ms["direct"] / ms["tiled"], 2),
                   "direct_over_plain": round(ms["direct"] / ms["plain"], 2),
                   "mask_cells_direct_vs_tiled_differing": same,
                   "paper_workstation_s": {"ca_cfar": PAPER_TABLE1_S[(g, b)][0],
                                           "ii_ca_cfar": PAPER_TABLE1_S[(g, b)][1]}}
            log(json.dumps(row))
            rows.append(row)
        del x, mask, masks
        torch.cuda.empty_cache()
    return {"table1": rows, "note": "direct = no integral image (each cell sums its window); tiled/plain = "
                                    "integral-image forms; paper times are a different machine and map size"}


def detections_bench(steps=10, warmup=2):
    """What the detector hands on, on the 16384 x 16384 FP32 map of the
    precision workload: the TILED detector, then the detection list (count
    pass + write pass) and the bit-packed mask, each timed with HIP events on
    one stream; bytes a host copy of each output would move."""
    import torch
    from paper_2012_11077_amd import cfar2d as C
    from paper_2012_11077_amd import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    spec = synth.config2()
    x = torch.from_numpy(synth.generate(spec)).to(dev)
    mask = torch.empty(x.shape, dtype=torch.uint8, device=dev)
    R, F = x.shape
    m = C.make_map(x, spec.window, mask)
    ws = torch.empty(C.workspace_bytes([m], C.TILED), dtype=torch.uint8, device=dev)
    wsd = torch.empty(C.lib().cfar_detections_workspace_bytes(C.ctypes.byref(m)), dtype=torch.uint8, device=dev)
    cnt = torch.zeros(1, dtype=torch.int64, device=dev)
    C.cfar2d(x, spec.window, C.TILED, mask=mask, ws=ws, stream=stream)
    C._check(C.lib().cfar_detections(C.ctypes.byref(m), None, 0, cnt.data_ptr(), wsd.data_ptr(), wsd.numel(),
                                     stream.cuda_stream))
    torch.cuda.synchronize()
    n_det = int(cnt.item())
    out = torch.empty(max(n_det, 1) * 3, dtype=torch.float64, device=dev)
    words = (F + 31) // 32
    bits = torch.empty((R, words), dtype=torch.int32, device=dev)
    steps_fn = {
        "detector": lambda: C.cfar2d(x, spec.window, C.TILED, mask=mask, ws=ws, stream=stream),
        "detection_list": lambda: C._check(C.lib().cfar_detections(
            C.ctypes.byref(m), out.data_ptr(), n_det, cnt.data_ptr(), wsd.data_ptr(), wsd.numel(),
            stream.cuda_stream)),
        "mask_pack": lambda: C._check(C.lib().cfar_mask_pack(C.ctypes.byref(m), bits.data_ptr(), words,
                                                             stream.cuda_stream)),
    }
    res = {}
    for name, fn in steps_fn.items():
        for _ in range(warmup):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(stream)
        for k in range(steps):
            fn()
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        res[name + "_ms"] = round(float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])), 4)
    cells = R * F
    # the list reads the mask twice (count and write passes) and writes 24 B per record
    res["detection_list_gbs"] = round((2 * cells + 24 * n_det) / (res["detection_list_ms"] / 1e3) / 1e9, 1)
    res["mask_pack_gbs"] = round((cells + cells / 8) / (res["mask_pack_ms"] / 1e3) / 1e9, 1)
    res.update({"map": "16384x16384 FP32, guard 4, training 24, Pfa 1e-5, seed 2", "detections": n_det,
                "host_bytes": {"dense_mask": cells, "packed_mask": R * words * 4, "detection_list": 24 * n_det}})
    return res


def mapbuild_bench(steps=10, warmup=2):
    """Building the map from raw records (cfar_map_build) then the TILED
    detector, timed with HIP events on one stream: a record of the paper's
    size (600 traces x 1024 samples) and a long one (4000 x 16384).  Table
    II's SBC times of the same steps are context (another machine)."""
    import torch
    from paper_2012_11077_amd import cfar2d as C
    from paper_2012_11077_amd import synth
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    rows = []
    for N, M in ((600, 1024), (4000, 16384)):
        spec = synth.RawSpec(n_traces=N, n_samples=M, target_bin=M * 2 // 3, seed=(12, N))
        raw = torch.from_numpy(synth.generate_raw(spec)).to(dev)
        win = (2, 2, 4, 4, 1e-4)
        res = {}
        for name, fn in (("map_build", lambda: C.build_map(raw, spec.fs_slow, stream=stream)),
                         ("map_build_and_cfar", lambda: C.cfar2d(C.build_map(raw, spec.fs_slow, stream=stream),
                                                                 win, C.TILED, stream=stream))):
            for _ in range(warmup):
                fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            ev[0].record(stream)
            for k in range(steps):
                fn()
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            res[name + "_ms"] = round(float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])), 4)
        k0, nb = C.map_bins(N, spec.fs_slow)
        res.update({"record": "%d traces x %d samples FP32" % (N, M), "band_bins": nb,
                    "raw_gbs": round(N * M * 4 / (res["map_build_ms"] / 1e3) / 1e9, 1)})
        log(json.dumps(res))
        rows.append(res)
    return {"mapbuild": rows, "paper_sbc_s": {"signal_processing_fast_time": 12.29,
                                              "signal_processing_slow_time": 16.37, "ii_ca_cfar": 1.17},
            "note": "times include allocations of the map and workspace by the Python binding"}


def serve_bench(seconds, seed=4, n_streams=16, log_every=5.0, packed=False):
    """The serving workload: n_streams simulated drone streams, each emitting
    frames of its own fixed size at Poisson rate 50 Hz, submitted from
    page-locked host memory (cfar_host_alloc) to the library's server (continuous batching over 4 HIP
    streams, admission by device memory); latency is frame arrival (its
    scheduled Poisson time) to the mask back in host memory (packed: the
    bit-packed mask, an eighth of the bytes)."""
    import threading
    import torch
    from paper_2012_11077_amd import cfar2d as C
    from paper_2012_11077_amd import synth
    streams = synth.config4_streams(n_streams, seed)
    rng = np.random.default_rng(seed)
    frames_per_stream, masks_per_stream = 4, 16
    frames, free_masks = [], []
    for st in streams:
        fr = []
        for j in range(frames_per_stream):
            sp = synth.stream_frame_spec(st, j)
            x = C.host_empty((sp.rows, sp.cols), torch.float32)   # page-locked (cfar_host_alloc)
            x.copy_(torch.from_numpy(synth.generate(sp)))
            fr.append((x, sp.window, sp.cells))
        frames.append(fr)
        shape = (st["rows"], (st["cols"] + 31) // 32) if packed else (st["rows"], st["cols"])
        free_masks.append([C.host_empty(shape, torch.int32 if packed else torch.uint8) for _ in range(masks_per_stream)])
    # merged Poisson arrival schedule
    arrivals = []
    for k, st in enumerate(streams):
        t = 0.0
        while True:
            t += rng.exponential(1.0 / st["rate_hz"])
            if t >= seconds:
                break
            arrivals.append((t, k))
    arrivals.sort()
    srv = C.Server(device_budget_bytes=4 << 30, max_inflight_frames=96, n_hip_streams=4, queue_depth=512,
                   max_batch_frames=32)
    lock = threading.Lock()
    pending = {}            # ticket -> (arrival_ns, stream, mask, cells)
    lat_ms, done_cells = [], [0]
    stop = [False]

    def poller():
        while True:
            cs = srv.poll(256, 20000)
            with lock:
                for c in cs:
                    arr, k, m, cells = pending.pop(c.ticket)
                    if c.status == C.CFAR_OK:
                        lat_ms.append((c.t_done_ns - arr) / 1e6)
                        done_cells[0] += cells
                    free_masks[k].append(m)
                if stop[0] and not pending:
                    return

    th = threading.Thread(target=poller, daemon=True)
    th.start()
    t0 = time.monotonic_ns()
    eagain = waited = 0
    next_log = log_every
    fi = [0] * len(streams)
    for (ta, k) in arrivals:
        arr_ns = t0 + int(ta * 1e9)
        now = time.monotonic_ns()
        if arr_ns > now:
            time.sleep((arr_ns - now) / 1e9)
        if ta >= next_log:
            log("serving: %.0f s, %d frames done" % (ta, len(lat_ms)))
            next_log += log_every
        x, win, cells = frames[k][fi[k] % frames_per_stream]
        fi[k] += 1
        while True:
            with lock:
                m = free_masks[k].pop() if free_masks[k] else None
            if m is not None:
                break
            waited += 1
            time.sleep(0.0002)
        while True:
            with lock:
                t = srv.submit(x, win, m, tag=k)
                if t is not None:
                    pending[t] = (arr_ns, k, m, cells)
                    break
            eagain += 1
            time.sleep(0.0002)
    srv.shutdown(drain=True)
    t_end = time.monotonic_ns()
    with lock:
        stop[0] = True
    th.join(timeout=60)
    st = srv.stats()
    srv.close()
    wall = (t_end - t0) / 1e9
    return {"seconds": round(wall, 2), "streams": n_streams, "rate_hz_per_stream": 50.0, "packed_masks": packed,
            "frame_sizes": "%dx%d .. %dx%d FP32" % (streams[0]["rows"], streams[0]["cols"], streams[-1]["rows"],
                                                   streams[-1]["cols"]),
            "frames": len(lat_ms), "failed": int(st.failed), "batches": int(st.batches),
            "mean_frames_per_batch": round(len(lat_ms) / max(1, int(st.batches)), 2),
            "p50_ms": round(percentile(lat_ms, 50), 3) if lat_ms else None,
            "p99_ms": round(percentile(lat_ms, 99), 3) if lat_ms else None,
            "max_ms": round(max(lat_ms), 3) if lat_ms else None,
            "cells_per_s": done_cells[0] / wall, "eagain": eagain, "mask_waits": waited,
            "device_bytes_peak": int(st.device_bytes_peak)}


def build_workload(name):
    from paper_2012_11077_amd import synth
    if name == "batched":
        specs = synth.config3_specs()
        desc = ("uneven batch: 512 FP32 maps, rows U[200,4096] x cols U[64,2048], Exp clutter mean "
                "log-U[0.1,10], 0-20 targets at 10-25 dB, guard 1-4 and training 4-24 per axis, "
                "Pfa in {1e-3,1e-4,1e-6}, seed 3")
    elif name == "precision":
        specs = [synth.config2()]
        desc = ("one 16384x16384 FP32 map, log-normal clutter sigma 2, 1000 targets at 8-30 dB, "
                "guard 4x4, training 24x24, Pfa 1e-5, seed 2")
    elif name == "plain_scale":
        specs = [synth.config1()]
        desc = ("one 8192x8192 FP64 map, Exp clutter on a 0-20 dB range ramp, 200 targets at 10-25 dB, "
                "guard 3x3, training 16x16, Pfa 1e-6, seed 1")
    elif name == "small":
        specs = [synth.config0()]
        desc = "one 512x256 FP64 map, Exp(1) clutter, 5 targets at 15 dB, guard 2x2, training 8x8, Pfa 1e-4"
    else:
        raise SystemExit("unknown workload %r" % name)
    return specs, desc


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "precision", "plain_scale", "small"])
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + steps of the tiled form only (for rocprofv3)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device 3 times (the counter scale of rocprofv3 FETCH_SIZE "
                         "and WRITE_SIZE)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving run (prints its JSON)")
    ap.add_argument("--mapbuild", action="store_true",
                    help="only the map-building timing (raw record -> map -> CA-CFAR)")
    ap.add_argument("--detections", action="store_true",
                    help="only the detection-list and packed-mask timing on the 16384^2 FP32 map")
    ap.add_argument("--table1", action="store_true",
                    help="only the Table I comparison: DIRECT vs TILED vs PLAIN per (guard, background) setting")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the serving run (16 Poisson streams at 50 Hz); 0 skips it")
    ap.add_argument("--packed-serve-seconds", type=float, default=10.0,
                    help="length of the serving run with bit-packed masks; 0 skips it")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the precision report (16384^2 FP32 map against the oracle)")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="write the traffic file from rocprofv3 --pmc output directories and exit")
    args = ap.parse_args()
    if args.record_traffic:
        if args.workload not in TRAFFIC_FILES:
            raise SystemExit("traffic is recorded for the workloads %s" % sorted(TRAFFIC_FILES))
        record_traffic(*args.record_traffic, workload=args.workload,
                       command="rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -- python3 bench.py --profile-only "
                               "--workload %s; copy scale from bench.py --copy-probe" % args.workload)
        return

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the workload would shard by map; see the design notes). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2012_11077_amd import cfar2d as C
    from paper_2012_11077_amd import synth

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    if args.copy_probe:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)   # an elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 3}), flush=True)
        return
    C.lib()
    if args.serve_only:
        print(json.dumps(serve_bench(args.serve_seconds)), flush=True)
        return
    if args.table1:
        print(json.dumps(table1_bench()), flush=True)
        return
    if args.detections:
        print(json.dumps(detections_bench()), flush=True)
        return
    if args.mapbuild:
        print(json.dumps(mapbuild_bench()), flush=True)
        return

    specs, desc = build_workload(args.workload)
    log("generating %d maps" % len(specs))
    t0 = time.perf_counter()
    arrays = [synth.generate(s) for s in specs]
    xs = [torch.from_numpy(a).to(dev) for a in arrays]
    torch.cuda.synchronize()
    log("generated + uploaded in %.1f s" % (time.perf_counter() - t0))
    cells = sum(s.cells for s in specs)
    in_bytes = sum(a.nbytes for a in arrays)
    elem = arrays[0].dtype.itemsize
    wins = [s.window for s in specs]

    # ---- chosen form: fused tiled, persistent launch, graph replay -------------
    masks = [torch.empty(x.shape, dtype=torch.uint8, device=dev) for x in xs]
    batch = C.Batch(xs, wins, C.TILED, masks=masks)
    flags = 0 if args.no_graph else C.BATCH_GRAPH
    # a stream of our own (default priority): the library captures and
    # replays its graph, and forks kernel classes, only on a non-null stream
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    for _ in range(args.warmup):
        batch.run(flags, stream=stream)
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        batch.run(flags, stream=stream)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    ms_per_step = evs[0].elapsed_time(evs[-1]) / args.steps
    value = cells / (ms_per_step / 1e3)
    log("tiled: %.3f ms/step, %.3e cells/s (wall %.3f ms/step)" % (ms_per_step, value, wall / args.steps * 1e3))

    if args.profile_only:
        print(json.dumps({"profile_only": True, "ms_per_step": ms_per_step}))
        return

    # ---- dominant kernel alone: HIP events around the persistent kernel ----------
    C.timing_enable(True)
    kms = []
    for _ in range(max(5, min(args.steps, 20))):
        batch.run(0, stream=stream)
        kms.append(C.timing_read())
    C.timing_enable(False)
    kernel_ms = float(np.mean(kms))
    alg_bytes = in_bytes + cells  # map read once + uint8 mask written once
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "fused_kernel", "kernel_ms": round(kernel_ms, 4),
            "alg_bytes_per_cell": round(alg_bytes / cells, 3)}
    tr = measured_traffic(args.workload)
    if tr and tr.get("workload") == args.workload:
        roof["traffic"] = tr["bytes_per_launch"]
        roof["traffic_unit"] = "bytes/launch"
        roof["traffic_per_cell"] = round(tr["bytes_per_launch"] / cells, 3)
    log("kernel %.3f ms -> %.1f GB/s algorithmic (%.1f%% of HBM peak)" % (kernel_ms, achieved, 100 * achieved / HBM_PEAK_GBS))

    # ---- plain per-map FP64 form on the same maps, compared at equal mask -------
    plain = None
    if not args.no_plain:
        pmasks = [torch.empty(x.shape, dtype=torch.uint8, device=dev) for x in xs]
        pbatch = C.Batch(xs, wins, C.PLAIN, masks=pmasks)
        pbatch.run(0, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.plain_steps):
            pbatch.run(0, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / args.plain_steps
        diff = sum(int((a != b).sum().item()) for a, b in zip(masks, pmasks))
        plain = {"ms_per_step": round(pms, 3), "cells_per_s": cells / (pms / 1e3),
                 "mask_cells_differing_from_tiled": diff}
        log("plain: %.3f ms/step (%d mask cells differ from tiled)" % (pms, diff))

    gpu_masks = [m.cpu().numpy() for m in masks]

    serving = serving_packed = None
    if args.serve_seconds > 0:
        log("serving run, %.0f s" % args.serve_seconds)
        serving = serve_bench(args.serve_seconds)
        log("serving: p50 %s ms, p99 %s ms, %d frames" % (serving["p50_ms"], serving["p99_ms"], serving["frames"]))
        if args.packed_serve_seconds > 0:
            serving_packed = serve_bench(args.packed_serve_seconds, packed=True)
            log("serving, packed masks: p50 %s ms, p99 %s ms" % (serving_packed["p50_ms"], serving_packed["p99_ms"]))

    precision = None
    if args.workload == "batched" and not args.no_precision:
        log("precision form report (16384^2 FP32 against the oracle)")
        precision = precision_report()
        log("precision: %s" % json.dumps(precision))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, whole workload)")
        cpu = cpu_baseline(specs, arrays, gpu_masks)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "maps": len(specs), "cells": cells,
                   "storage_dtype": str(arrays[0].dtype), "form": "tiled (fused, FP64 carries)",
                   "graph": not args.no_graph, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "latency_ms": ({"p50": serving["p50_ms"], "p99": serving["p99_ms"],
                        "what": "serving: frame arrival to mask in host memory, 16 Poisson streams at 50 Hz"}
                       if serving else None),
        "launch_latency_ms": {"p50": round(percentile(step_ms, 50), 4), "p99": round(percentile(step_ms, 99), 4),
                              "what": "per batched launch, back-to-back"},
        "serving": serving,
        "serving_packed_masks": serving_packed,
        "plain_form": plain,
        "speedup_vs_plain": (round(plain["ms_per_step"] / ms_per_step, 3) if plain else None),
        "precision_form": precision,
        "effective_hbm_frac": round((in_bytes + cells) / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
