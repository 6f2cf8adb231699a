"""Autotuner for the line-solver launch shape.

For one (bands, n, precision, grid shape, axis) it times every valid choice of
  * partitions    -- workgroups per line (the two-level split of Sec. 3-4 with
    workgroups as partitions; FP64 lines of 1024 rows or more),
  * rows_per_lane -- where the reduction switches from registers (generalized
    PCR inside a lane, ceil(log2(rows_per_lane - r)) levels) to LDS (block
    PCR across lanes, log2(lanes) levels),
  * lines_per_wg  -- lines per workgroup (tile width),
  * block_barriers -- wavefront-local or workgroup-wide lane exchanges,
  * x_staging     -- unit-stride lines read directly or through an LDS tile,
  * interior      -- lane interiors by generalized PCR or banded elimination
                     (the latter for 8, 12 or 16 rows per lane),
  * tile_order    -- strided lines: tiles in launch order or grouped by XCD,
with HIP events on the launch stream, and returns the fastest.  Results are
cached in a JSON file keyed by the problem so a process tunes once.
"""
import json
import os

import numpy as np
import torch

from . import cb

ROWS = (4, 6, 8, 12, 16)
LINES = (0, 1, 2, 4, 8, 16, 32, 64)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "cb_tune.json")


def _key(bands, n, precision, shape, axis, fused):
    return "r%d|n%d|%s|%s|ax%d|%s|%s" % ((len(bands) - 1) // 2, n, precision, "x".join(map(str, shape)), axis,
                                        "fused" if fused else "solve", ",".join("%.17g" % b for b in bands))


PARTS = (2, 4, 8, 16)


def candidates(bands, n, precision, strided=None):
    """Launch choices to time.  `strided` True: rows are strided (x_staging is
    moot; both tile orders are tried); False: unit-stride rows; None: both."""
    out = []
    xss = (0,) if strided else (1, 2)
    orders = (1, 2) if strided else (0,)
    if precision == "fp64" and n >= 1024:
        for P in PARTS:
            for rpl in (8, 16):
                try:
                    cb.Plan(bands, n, partitions=P, rows_per_lane=rpl, host_only=True).close()
                except cb.CbError:
                    continue
                for w in (0, 2, 4, 8):
                    for xs in xss:
                        out.append(dict(partitions=P, rows_per_lane=rpl, lines_per_wg=w, block_barriers=0,
                                        x_staging=xs, interior=1, tile_order=0))
    for rpl in ROWS:
        try:
            p = cb.Plan(bands, n, precision=precision, rows_per_lane=rpl, host_only=True)
        except cb.CbError:
            continue
        L = p.info()["lanes"]
        p.close()
        for w in LINES:
            if w and w * L > 1024:
                continue
            for bb in (0, 1):
                for xs in xss:
                    for it in ((1, 2) if rpl in (8, 12, 16) else (1,)):
                        for to in orders:
                            out.append(dict(partitions=1, rows_per_lane=rpl, lines_per_wg=w, block_barriers=bb,
                                            x_staging=xs, interior=it, tile_order=to))
    return out


def _time(fn, reps, stream):
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(bands, n, f, axis, stencil=None, precision="fp64", refine_iters=0, reps=5, cache=DEFAULT_CACHE,
         max_candidates=None, one_partition=False):
    """Return (best_kwargs, table) for solving/deriving along `axis` of tensor f
    (`one_partition`: only P = 1 plans, e.g. for batched launches)."""
    key = _key(bands, n, precision, tuple(f.shape), axis, stencil is not None) + ("|p1" if one_partition else "")
    db = {}
    if cache and os.path.exists(cache):
        try:
            db = json.load(open(cache))
        except (OSError, ValueError):
            db = {}
    if key in db:
        return db[key]["best"], db[key]["table"]
    stream = torch.cuda.current_stream()
    out = torch.empty_like(f)
    table = []
    cands = candidates(bands, n, precision, strided=f.stride(2 - axis) != 1)
    if one_partition:
        cands = [c for c in cands if c["partitions"] == 1]
    if max_candidates:
        cands = cands[:max_candidates]
    for c in cands:
        try:
            p = cb.Plan(bands, n, precision=precision, refine_iters=refine_iters, **c)
        except cb.CbError:
            continue
        if stencil is not None:
            fn = lambda: cb.apply_derivative(p, stencil, f, axis, out=out, stream=stream)
        else:
            fn = lambda: cb.solve(p, f, axis, out=out, stream=stream)
        try:
            ms = _time(fn, reps, stream)
        except cb.CbError:
            p.close()
            continue
        table.append(dict(c, ms=ms))
        p.close()
    best = min(table, key=lambda r: r["ms"])
    best = {k: best[k] for k in ("partitions", "rows_per_lane", "lines_per_wg", "block_barriers", "x_staging",
                                 "interior", "tile_order")}
    if cache:
        db[key] = {"best": best, "table": table}
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp%d" % os.getpid()
        json.dump(db, open(tmp, "w"), indent=1)
        os.replace(tmp, cache)
    return best, table


def tuned_plan(bands, n, f, axis, stencil=None, precision="fp64", refine_iters=0, **kw):
    best, _ = tune(bands, n, f, axis, stencil, precision, refine_iters, **kw)
    return cb.Plan(bands, n, precision=precision, refine_iters=refine_iters, **best)
