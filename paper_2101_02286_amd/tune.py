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

tune_batch() tunes a batched launch as a whole: a batch runs one launch per
kernel class, so a choice that is fastest for one item alone can split the
batch into more classes and slow it down.  It starts from the automatic plans
and, one group of items sharing a matrix and row layout at a time, keeps a
choice only when the whole batch gets faster.
"""
import collections
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


BATCH_ROWS = (4, 6, 8, 12, 16, 32)


def batch_candidates(bands, n, precision, refine_iters=0, strided=False):
    """Plan choices that change a batched launch of lines of n rows: rows per
    lane, interior solve, and the lane exchanges (unit-stride rows) or the
    tile order (strided rows).  Lines per workgroup and unit-stride staging
    are the batch's own choice and are not searched."""
    out = []
    for rpl in BATCH_ROWS:
        try:
            cb.Plan(bands, n, precision=precision, refine_iters=refine_iters, rows_per_lane=rpl,
                    host_only=True).close()
        except cb.CbError:
            continue
        interiors = (2,) if rpl == 32 else ((1, 2) if rpl in (8, 12, 16) else (1,))
        for it in interiors:
            for v in ((1, 2) if strided else (0, 1)):
                c = dict(rows_per_lane=rpl, interior=it)
                c.update(dict(tile_order=v) if strided else dict(block_barriers=v))
                out.append(c)
    return out


def tune_batch(items, precision="fp64", refine_iters=0, reps=5, max_ctas=-1, min_gain=0.02, stream=None,
               max_candidates=None):
    """Tune the plans of a batched launch by its whole-batch time.

    items: (bands, stencil or None, f, out, axis) tuples; items with the same
    bands, line length and row layout (unit stride or strided) share a plan
    (a group).  Starting from the automatic plans, for each group in order of
    decreasing unknowns, every choice of batch_candidates() is timed in the
    whole batch (median of `reps` launches) and kept when it is faster than
    the best so far by more than `min_gain`.

    Returns (plans, choices, result): plans[i] is item i's plan (shared
    objects within a group), choices maps a group's description to the plan
    arguments kept ({} = automatic), and result holds the automatic and tuned
    batch times in ms and the number of timed candidates."""
    stream = stream or torch.cuda.current_stream()
    groups = collections.OrderedDict()
    for i, (bands, st, f, out, ax) in enumerate(items):
        n = f.shape[2 - ax]
        key = (tuple(float(b) for b in bands), n, f.stride(2 - ax) != 1)
        groups.setdefault(key, []).append(i)

    def make(key, kw):
        return cb.Plan(list(key[0]), key[1], precision=precision, refine_iters=refine_iters, **kw)

    plans = {k: make(k, {}) for k in groups}
    choice = {k: {} for k in groups}
    ws = [None]

    def batch_ms(pl):
        b = cb.Batch([(pl[k], items[i][1], items[i][2], items[i][3], items[i][4])
                      for k, idx in groups.items() for i in idx], stream=stream, workspace=ws[0])
        ws[0] = b.ws
        return _time(lambda: b.launch(max_ctas, stream), reps, stream)

    base = best = batch_ms(plans)
    timed = 0
    order = sorted(groups, key=lambda k: -sum(items[i][2].numel() for i in groups[k]))
    for k in order:
        cands = batch_candidates(list(k[0]), k[1], precision, refine_iters, strided=k[2])
        if max_candidates:
            cands = cands[:max_candidates]
        for c in cands:
            try:
                p = make(k, c)
            except cb.CbError:
                continue
            trial = dict(plans)
            trial[k] = p
            try:
                ms = batch_ms(trial)
            except cb.CbError:
                p.close()
                continue
            timed += 1
            if ms < best * (1.0 - min_gain):
                plans[k].close()
                plans[k], choice[k], best = p, c, ms
            else:
                p.close()
    final = batch_ms(plans)
    per_item = [None] * len(items)
    for k, idx in groups.items():
        for i in idx:
            per_item[i] = plans[k]
    desc = {"n%d %s r%d" % (k[1], "strided" if k[2] else "unit-stride", (len(k[0]) - 1) // 2): choice[k]
            for k in groups}
    return per_item, desc, {"automatic_ms": base, "tuned_ms": final, "candidates_timed": timed}
