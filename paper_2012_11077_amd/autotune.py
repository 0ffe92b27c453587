"""Autotuner of the TILED form's tile plans.

    python -m paper_2012_11077_amd.autotune [--out paper_2012_11077_amd/plan_table.txt] [--quick]

For every shape family (FP32/FP64 x map width x window half-width x map
height) it builds a batch of synthetic maps of that family, times each
candidate plan (columns per lane k, rows per work unit, LDS ring budget) on
the GPU with the library's own kernel timing, and writes the fastest plan of
every family as one rule of a plan table (the format cfar_plan_load reads:
``dtype cols_lo cols_hi rows_lo rows_hi hf_lo hf_hi hr_lo hr_hi k rows_per_unit
ring_bytes``).  Maps that match no rule keep the library's built-in cost
model.  A plan changes speed only: every plan computes the same detector.
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2012_11077_amd import cfar2d as C  # noqa: E402
from paper_2012_11077_amd import synth  # noqa: E402

# family buckets (inclusive ranges)
COLS = [(1, 127), (128, 255), (256, 511), (512, 1023), (1024, 2047), (2048, 8191), (8192, 1 << 30)]
HALF = [(0, 4), (5, 12), (13, 28), (29, 247)]
ROWS = [(1, 1023), (1024, 1 << 30)]
CANDIDATES = [(k, rs, ring) for k in (2, 4) for rs in (64, 128) for ring in (0, 12288, 24576)]
TARGET_CELLS = 24_000_000


def family_maps(dtype, cols, half, rows, seed):
    """Synthetic maps of one family, enough cells to time a launch well."""
    rng = np.random.default_rng(seed)
    c_lo, c_hi = cols[0], min(cols[1], 16384)
    r_lo, r_hi = max(rows[0], 64), min(rows[1], 8192)
    h_lo, h_hi = half[0], min(half[1], 60)
    specs, cells = [], 0
    while cells < TARGET_CELLS and len(specs) < 512:
        R = int(rng.integers(r_lo, r_hi + 1))
        F = int(rng.integers(c_lo, c_hi + 1))
        h = int(rng.integers(max(h_lo, 1), h_hi + 1))
        g = max(0, min(4, h // 5))
        specs.append(synth.MapSpec(R, F, dtype, "exp", 1.0, n_targets=2, guard_r=g, guard_f=g,
                                   train_r=max(h - g, 1), train_f=max(h - g, 1), pfa=1e-4,
                                   seed=(int(seed), len(specs))))
        cells += R * F
    return specs


def rule(dtype, cols, half, rows, k, rs, ring):
    return "%s %d %d %d %d %d %d %d %d %d %d %d" % (dtype, cols[0], cols[1], rows[0], rows[1], half[0], half[1],
                                                   half[0], half[1], k, rs, ring)


def time_batch(xs, wins, reps):
    import torch
    side = torch.cuda.Stream()
    masks = [torch.empty(x.shape, dtype=torch.uint8, device=x.device) for x in xs]
    b = C.Batch(xs, wins, C.TILED, masks=masks)
    b.run(0, stream=side)
    torch.cuda.synchronize()
    C.timing_enable(True)
    ts = []
    for _ in range(reps):
        b.run(0, stream=side)
        ts.append(C.timing_read())
    C.timing_enable(False)
    return float(np.median(ts))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "plan_table.txt"))
    ap.add_argument("--dtypes", default="f32,f64")
    ap.add_argument("--quick", action="store_true", help="f32 only, fewer families (a smoke run)")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the autotuner times plans on the GPU")
    dev = "cuda:0"
    dtypes = ["f32"] if args.quick else args.dtypes.split(",")
    cols = COLS[2:5] if args.quick else COLS
    rules, log = [], []
    with tempfile.TemporaryDirectory() as td:
        probe = os.path.join(td, "probe.txt")
        for n_fam, (dt, cb, hb, rb) in enumerate(itertools.product(dtypes, cols, HALF, ROWS)):
            specs = family_maps(dt, cb, hb, rb, seed=1000 + n_fam)
            xs = [torch.from_numpy(synth.generate(s)).to(dev) for s in specs]
            wins = [s.window for s in specs]
            best = None
            for (k, rs, ring) in CANDIDATES:
                with open(probe, "w") as f:
                    f.write(rule(dt, cb, hb, rb, k, rs, ring) + "\n")
                try:
                    C.plan_load(probe)
                    ms = time_batch(xs, wins, args.reps)
                except C.CfarError:
                    continue          # plan not valid for some map of the family
                if best is None or ms < best[0]:
                    best = (ms, k, rs, ring)
            C.plan_load(None)
            if best is None:
                continue
            cells = sum(s.cells for s in specs)
            rules.append(rule(dt, cb, hb, rb, best[1], best[2], best[3]))
            log.append({"dtype": dt, "cols": cb, "half": hb, "rows": rb, "maps": len(specs), "cells": cells,
                        "best": {"k": best[1], "rs": best[2], "ring": best[3], "ms": round(best[0], 4),
                                 "gcells_s": round(cells / best[0] / 1e6, 1)}})
            print(json.dumps(log[-1]), flush=True)
            del xs
            torch.cuda.empty_cache()
    with open(args.out, "w") as f:
        f.write("# Tile plans chosen by paper_2012_11077_amd/autotune.py on %s, %s\n"
                % (torch.cuda.get_device_name(0), time.strftime("%Y-%m-%d")))
        f.write("# dtype cols_lo cols_hi rows_lo rows_hi hf_lo hf_hi hr_lo hr_hi k rows_per_unit ring_bytes\n")
        for r in rules:
            f.write(r + "\n")
    print("wrote %d rules to %s" % (len(rules), args.out), flush=True)


if __name__ == "__main__":
    main()
