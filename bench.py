"""Benchmark: cyclic compact-banded PCR solves on one MI355X.

Default workload (the headline): a 512^3 periodic FP64 grid, sixth-order
compact first derivative (cyclic tridiagonal, alpha = 1/3) fused with its
right-hand-side stencil, along x, y and z.  One step = the three directions
(3 x 134,217,728 solved unknowns).  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  `value` is GDOF/s (solved unknowns per
second); `roofline` uses the algorithmic 16 bytes per unknown (read f, write
f') of the dominant kernel launch, timed with HIP events on the launch stream.
The same line then summarises the other workloads under their own keys
(medians of HIP-event timed launches, inputs resident in HBM): a device copy
(the practical HBM ceiling, `roofline.frac_of_copy`), plain cb_solve along
x/y/z of the 512^3 grid, the 32^3 and 256^3 grids (derivative and
interpolation), 4096 lines of n = 8192 in 16 workgroup partitions with the
16/15 and 8/7 partition comparison, the 512^3 pentadiagonal derivative, the
batch of 12 uneven grids (FP64 and FP32 + refinement) and the served request
stream (p50/p99 latency, GDOF/s).  --no-extras prints the headline alone.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2101_02286_amd import cb, schemes, synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_DOF = 16
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE (scaled
# by what the counters read for a plain copy of known size); reported only
# while the kernel sources hash to what was profiled
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_line_deriv6_512cubed_hbm_bytes.txt")


def csrc_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2101_02286_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h", ".cpp")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()


def measured_traffic(group):
    """HBM bytes per launch of kernel group `group` from the committed counter summary, or None."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        if ":" in ln and not ln.startswith((" ", "#")):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("csrc_sha256") != csrc_hash():
        return None
    v = kv.get("bytes_per_launch " + group)
    return int(float(v)) if v else None


def kernel_group(plan, axis):
    """Name of the line-kernel instance a launch along `axis` uses (unit-stride or strided layout)."""
    i = plan.info()
    if axis == 0:
        return "unit-stride/r%d/rows%d/%s" % (i["r"], i["rows_per_lane"],
                                              "elim" if i["interior_elimination"] else "pcr")
    return "strided/r%d/rows%d/%s" % (i["r"], i["rows_per_lane_strided"],
                                      "elim" if i["interior_elimination_strided"] else "pcr")


def scheme_stencil(name, n):
    """cb.Stencil of a named compact scheme's right-hand side for lines of n points."""
    return cb.Stencil(*schemes.stencil(name, n))


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform string."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(f_dev, bands, stencils, seconds=10.0, runs=5):
    """The FP64 oracle on the host cores, over a bounded sample of the same work:
    the fused derivative along x and y of z-slabs of the grid and along z of
    y-slabs.  `runs` timed runs of about seconds/runs each; the median rate."""
    import oracle
    f = f_dev.cpu().numpy()
    nz, ny, nx = f.shape
    slab = max(1, nz // 8)
    srcs = [np.ascontiguousarray(f[:slab]), np.ascontiguousarray(f[:slab]),
            np.ascontiguousarray(f[:, :max(1, ny // 8), :])]
    rates, t_all = [], 0.0
    for _ in range(runs):
        t_run, dof = 0.0, 0
        while t_run < seconds / runs:
            for axis in range(3):
                st = stencils[axis]
                t0 = time.perf_counter()
                oracle.apply_axis(srcs[axis], axis, bands, st.lo, st.coefs)
                t_run += time.perf_counter() - t0
                dof += srcs[axis].size
        rates.append(dof / t_run / 1e9)
        t_all += t_run
    return {"value": round(float(np.median(rates)), 4), "unit": "GDOF/s", "cores": oracle.num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "runs_gdofs": [round(r, 4) for r in rates],
            "sample": "FP64 oracle (banded LU + Woodbury, OpenMP over lines): fused derivative along x and y of "
                      "%d z-planes and along z of %d y-rows of the %d^3 grid; median of %d runs, %.1f s in all"
                      % (slab, max(1, ny // 8), nx, runs, t_all)}


def headline(args):
    dev = torch.device("cuda:0")
    n = args.n
    shape = (n, n, n)
    bands = schemes.bands("tri6")
    st = scheme_stencil("tri6", n)
    f, _ = synth.random_modes(shape, seed=0, device=dev)
    if not args.tune:  # the plans' automatic launch shape
        plans = [cb.Plan(bands, n)] * 3
        tuned = None
    else:  # autotuned launch shape per direction (rows per lane, lines per workgroup, barriers)
        from paper_2101_02286_amd import tune
        tuned, plans = {}, []
        for ax in range(3):
            best, _ = tune.tune(bands, n, f, ax, stencil=st, reps=3, cache=None)
            tuned["xyz"[ax]] = best
            plans.append(cb.Plan(bands, n, **best))
    outs = [torch.empty_like(f) for _ in range(3)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        for ax in range(3):
            cb.apply_derivative(plans[ax], st, f, ax, out=outs[ax], stream=stream)
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        for ax in range(3):
            ev[k][ax][0].record(stream)
            cb.apply_derivative(plans[ax], st, f, ax, out=outs[ax], stream=stream)
            ev[k][ax][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dur = np.array([[ev[k][ax][0].elapsed_time(ev[k][ax][1]) for ax in range(3)] for k in range(args.steps)])
    dof = n ** 3
    per_dir_ms = dur.mean(axis=0)
    step_ms = wall * 1e3 / args.steps
    value = 3 * dof / (wall / args.steps) / 1e9
    # dominant kernel: the line-kernel instance with the largest time per step
    groups = {}
    for ax in range(3):
        groups.setdefault(kernel_group(plans[ax], ax), []).append(ax)
    dom = max(groups, key=lambda g: sum(per_dir_ms[ax] for ax in groups[g]))
    dom_ms = float(np.mean([per_dir_ms[ax] for ax in groups[dom]]))  # average launch duration
    achieved = BYTES_PER_DOF * dof / (dom_ms * 1e-3) / 1e9
    lat = dur.reshape(-1)
    # the same launches with the arithmetic left out (cb_copy_lines): the
    # ceiling of each direction's own access pattern
    copy_ms = []
    for ax in range(3):
        copy_ms.append(_median_ms(lambda: cb.copy_lines(plans[ax], f, ax, out=outs[ax], stream=stream),
                                  args.steps, args.warmup, stream))
    dom_copy_ms = float(np.mean([copy_ms[ax] for ax in groups[dom]]))
    res = {
        "metric": "GDOF/s (solved unknowns per second), 512^3 cyclic tridiagonal compact derivative x/y/z",
        "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (8 seeded random Fourier modes, seed 0)",
        "config": {"workload": "%d^3 periodic grid, sixth-order compact first derivative (cyclic tridiagonal "
                               "alpha=1/3) fused with its stencil, along x, y, z" % n,
                   "n": n, "lines_per_direction": n * n, "partitions": 1,
                   "launch": {k: {"rows_per_lane": (p.info()["rows_per_lane"] if k == "x"
                                                    else p.info()["rows_per_lane_strided"])}
                              for k, p in zip("xyz", plans)},
                   "autotuned": tuned},
        "per_direction_ms": {k: round(float(v), 4) for k, v in zip("xyz", per_dir_ms)},
        "per_direction_gdofs": {k: round(dof / (float(v) * 1e-3) / 1e9, 2) for k, v in zip("xyz", per_dir_ms)},
        "achieved_hbm_gbs_algorithmic": {k: round(BYTES_PER_DOF * dof / (float(v) * 1e-3) / 1e9, 1)
                                         for k, v in zip("xyz", per_dir_ms)},
        "solve_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                             "p99": round(float(np.percentile(lat, 99)), 4)},
        "copy_same_pattern": {k: {"ms": round(c, 4), "gbs": round(BYTES_PER_DOF * dof / (c * 1e-3) / 1e9, 1),
                                  "solve_over_copy_time": round(float(v) / c, 3)}
                              for k, c, v in zip("xyz", copy_ms, per_dir_ms)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                     "kernel": "k_line %s (%s)" % (dom, ", ".join("xyz"[ax] for ax in groups[dom])),
                     "avg_launch_ms": round(dom_ms, 4), "bytes_per_launch": BYTES_PER_DOF * dof,
                     "copy_same_pattern_gbs": round(BYTES_PER_DOF * dof / (dom_copy_ms * 1e-3) / 1e9, 1),
                     "frac_of_copy_same_pattern": round(dom_copy_ms / dom_ms, 4)},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(f, bands, [st, st, st], seconds=args.cpu_seconds)
    for p in set(plans):
        p.close()
    del f, outs
    torch.cuda.empty_cache()
    if not args.no_extras:
        # the other workloads, each summarised under its own key (a failing
        # leg reports its error and the others still run)
        steps, warm = 10, 2
        legs = (("copy_ceiling", lambda: leg_copy(1024, steps, warm)),
                ("solve_512", lambda: leg_solve(n, steps, warm)),
                ("small_grids", lambda: leg_small(steps, warm)),
                ("two_level_8192", lambda: leg_two_level(steps, warm)),
                ("penta10_512", lambda: leg_penta(n, steps, warm)),
                ("batched_12_grids", lambda: leg_batched(steps, warm)),
                ("served", lambda: leg_served(args.serve_requests, args.max_points)))
        for key, fn in legs:
            t0 = time.perf_counter()
            try:
                res[key] = fn()
            except Exception as e:  # noqa: BLE001 -- reported in the line, the headline stands
                res[key] = {"error": "%s: %s" % (type(e).__name__, e)}
            res[key]["leg_wall_s"] = round(time.perf_counter() - t0, 1)
            torch.cuda.empty_cache()
        cp = res["copy_ceiling"].get("gbs")
        if cp:
            res["roofline"]["copy_gbs"] = cp
            res["roofline"]["frac_of_copy"] = round(achieved / cp, 4)
    return res


def _median_ms(fn, steps, warmup, stream):
    dur, _ = _time_launches(fn, steps, warmup, stream)
    return float(np.median(dur))


def leg_solve(n, steps, warmup):
    """Plain cb_solve (b = stencil(f) precomputed) along x, y, z of the n^3 grid."""
    dev = torch.device("cuda:0")
    bands = schemes.bands("tri6")
    plan = cb.Plan(bands, n)
    st = scheme_stencil("tri6", n)
    f, _ = synth.random_modes((n, n, n), seed=0, device=dev)
    out = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    res = {}
    for ax in range(3):
        b = cb.rhs_stencil(st, f, ax)
        ms = _median_ms(lambda: cb.solve(plan, b, ax, out=out, stream=stream), steps, warmup, stream)
        res["xyz"[ax]] = {"ms": round(ms, 4), "gdofs": round(n ** 3 / (ms * 1e-3) / 1e9, 2)}
        del b
    plan.close()
    return {"workload": "%d^3 cyclic tridiagonal (alpha=1/3) cb_solve of b = stencil(f), per direction" % n,
            "per_direction": res}


def leg_copy(mib, steps, warmup):
    """A plain device copy (torch copy_) of `mib` MiB: the practical HBM ceiling."""
    dev = torch.device("cuda:0")
    a = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    ms = _median_ms(lambda: b.copy_(a), steps, warmup, stream)
    return {"workload": "device copy of %d MiB (read + write)" % mib, "ms": round(ms, 4),
            "gbs": round(2 * a.numel() * 8 / (ms * 1e-3) / 1e9, 1)}


def leg_small(steps, warmup):
    """32^3 x derivative and 256^3 derivative + collocated-to-staggered interpolation along x, y, z."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    res = {}
    for n, axes, kinds in ((32, (0,), ("deriv6",)), (256, (0, 1, 2), ("deriv6", "interp6_c2s"))):
        f, _ = synth.random_modes((n, n, n), seed=0, device=dev)
        out = torch.empty_like(f)
        for kind in kinds:
            if kind == "deriv6":
                bands, st = schemes.bands("tri6"), scheme_stencil("tri6", n)
            else:
                bands = schemes.bands("interp6")
                st = cb.Stencil(*schemes.stencil("interp6", n))
            plan = cb.Plan(bands, n)
            for ax in axes:
                ms = _median_ms(lambda: cb.apply_derivative(plan, st, f, ax, out=out, stream=stream), steps, warmup,
                                stream)
                res["%d^3 %s %s" % (n, kind, "xyz"[ax])] = {"ms": round(ms, 4),
                                                             "gdofs": round(n ** 3 / (ms * 1e-3) / 1e9, 2)}
            plan.close()
    return {"workload": "32^3 sixth-order derivative along x; 256^3 derivative and interpolation along x, y, z",
            "runs": res}


def leg_two_level(steps, warmup):
    """64x64 lines of n = 8192 with P = 16 workgroup partitions (cb_solve along x, y and z), and the
    one-GPU analogue of the power-of-two vs one-less partition comparison: 512-row partitions,
    P = 16 / 15 and 8 / 7 (n = 512 P), x lines."""
    dev = torch.device("cuda:0")
    bands = schemes.bands("tri6")
    stream = torch.cuda.current_stream()
    res = {}
    n, P = 8192, 16
    plan = cb.Plan(bands, n, partitions=P)
    plan32 = cb.Plan(bands, n, partitions=P, precision="fp32_refine")
    for ax in range(3):
        dims = [64, 64]
        dims.insert(ax, n)
        b = synth.random_uniform((dims[2], dims[1], dims[0]), seed=3, device=dev)
        x = torch.empty_like(b)
        ms = _median_ms(lambda: cb.solve(plan, b, ax, out=x, stream=stream), steps, warmup, stream)
        res["n8192_P16_" + "xyz"[ax]] = {"ms": round(ms, 4), "gdofs": round(b.numel() / (ms * 1e-3) / 1e9, 2)}
        if ax == 0:  # FP32 + refinement (automatic count) on the same lines, against the FP64 result
            x32 = torch.empty_like(b)
            ms32 = _median_ms(lambda: cb.solve(plan32, b, ax, out=x32, stream=stream), steps, warmup, stream)
            torch.cuda.synchronize()
            res["n8192_P16_x_fp32_refine"] = {
                "ms": round(ms32, 4), "gdofs": round(b.numel() / (ms32 * 1e-3) / 1e9, 2),
                "refine_iters": plan32.info()["refine_iters"],
                "max_rel_diff_vs_fp64": float(((x32 - x).abs().max() / x.abs().max()).item())}
    plan.close()
    plan32.close()
    scal = {}
    for P in (16, 15, 8, 7):
        n = 512 * P
        plan = cb.Plan(bands, n, partitions=P)
        b = synth.random_uniform((64, 64, n), seed=4, device=dev)
        x = torch.empty_like(b)
        ms = _median_ms(lambda: cb.solve(plan, b, 0, out=x, stream=stream), steps, warmup, stream)
        info = plan.info()
        scal["P%d" % P] = {"n": n, "ms": round(ms, 4), "gdofs": round(b.numel() / (ms * 1e-3) / 1e9, 2),
                           "pcr_steps": info["red_pcr_steps"], "detach_steps": info["red_detach_steps"]}
        plan.close()
    return {"workload": "4096 lines of n=8192, P=16 workgroup partitions, cb_solve per axis; 512-row partitions "
                        "at P = 16/15 and 8/7", "runs": res, "pow2_vs_one_less": scal}


def leg_penta(n, steps, warmup):
    """n^3 tenth-order pentadiagonal compact derivative (alpha=1/2, beta=1/20) along x, y, z."""
    dev = torch.device("cuda:0")
    bands = schemes.bands("penta10")
    st = scheme_stencil("penta10", n)
    plan = cb.Plan(bands, n)
    f, _ = synth.random_modes((n, n, n), seed=1, device=dev)
    out = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    res = {}
    for ax in range(3):
        ms = _median_ms(lambda: cb.apply_derivative(plan, st, f, ax, out=out, stream=stream), steps, warmup, stream)
        res["xyz"[ax]] = {"ms": round(ms, 4), "gdofs": round(n ** 3 / (ms * 1e-3) / 1e9, 2)}
    plan.close()
    return {"workload": "%d^3 tenth-order cyclic pentadiagonal compact derivative fused with its stencil" % n,
            "per_direction": res}


def _time_launches(fn, steps, warmup, stream):
    """Run fn() warmup + steps times; return per-launch HIP-event durations (ms) and wall seconds."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return np.array([a.elapsed_time(b) for a, b in evs]), wall


def mode_two_level(args):
    """n = 8192 lines (64 x 64 of them) split into P = 16 workgroup partitions."""
    dev = torch.device("cuda:0")
    n, P = 8192, 16
    bands = schemes.bands("tri6")
    plan = cb.Plan(bands, n, partitions=P)
    f, _ = synth.random_modes((64, 64, n), seed=3, device=dev)
    rhs = cb.rhs_stencil(scheme_stencil("tri6", n), f, 0)
    x = torch.empty_like(rhs)
    stream = torch.cuda.current_stream()
    dur, wall = _time_launches(lambda: cb.solve(plan, rhs, 0, out=x, stream=stream), args.steps, args.warmup, stream)
    dof = rhs.numel()
    ms = float(dur.mean())
    return {"metric": "GDOF/s, cyclic tridiagonal n=8192 two-level (P=16 workgroup partitions)",
            "value": round(dof / (ms * 1e-3) / 1e9, 3), "unit": "GDOF/s", "ms_per_solve": round(ms, 4),
            "hbm_gbs_algorithmic": round(16 * dof / (ms * 1e-3) / 1e9, 1),
            "hbm_gbs_moved": round(24 * dof / (ms * 1e-3) / 1e9, 1),
            "p50_ms": round(float(np.percentile(dur, 50)), 4), "p99_ms": round(float(np.percentile(dur, 99)), 4),
            "config": {"workload": "64x64 lines of n=8192, P=16", "partitions": P}, "dtype": "f64"}


def mode_penta_z(args):
    """512^3 tenth-order pentadiagonal compact derivative along z."""
    dev = torch.device("cuda:0")
    n = args.n
    bands = schemes.bands("penta10")
    st = scheme_stencil("penta10", n)
    plan = cb.Plan(bands, n)
    f, _ = synth.random_modes((n, n, n), seed=1, device=dev)
    out = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    res = {}
    for ax in range(3):
        dur, wall = _time_launches(lambda: cb.apply_derivative(plan, st, f, ax, out=out, stream=stream),
                                   args.steps, args.warmup, stream)
        ms = float(dur.mean())
        res["xyz"[ax]] = {"ms": round(ms, 4), "gdofs": round(n ** 3 / (ms * 1e-3) / 1e9, 2),
                          "hbm_gbs_algorithmic": round(16 * n ** 3 / (ms * 1e-3) / 1e9, 1)}
    return {"metric": "GDOF/s, %d^3 tenth-order pentadiagonal compact derivative" % n, "per_direction": res,
            "dtype": "f64", "config": {"workload": "%d^3, alpha=1/2 beta=1/20" % n}}


def batched_runs(variants, steps, warmup, batch_ctas=-1, tune=False, extras=True):
    """12 uneven periodic grids x 3 axes in one batched launch per kernel class, for each
    (key, precision, refine_iters) variant; with `extras` the persistent work-queue form and a
    graph replay of the same launches are timed too.  With `tune` the plans are tuned for the
    whole batch (tune.tune_batch, starting from the automatic plans) and the automatic batch
    time is reported beside the tuned one.  FP32 variants report their max relative difference
    to the FP64 outputs."""
    dev = torch.device("cuda:0")
    shapes = synth.grid_batch_shapes(seed=0, count=12)
    bands = schemes.bands("tri6")
    fields = []
    for gi, (nx, ny, nz) in enumerate(shapes):
        f, _ = synth.random_modes((nz, ny, nx), seed=gi, device=dev)
        fields.append(f)
    stencils = {}
    out = {}
    for key, prec, iters in variants:
        spec = []
        for f in fields:
            for ax in range(3):
                n = f.shape[2 - ax]
                if n not in stencils:
                    stencils[n] = scheme_stencil("tri6", n)
                spec.append((bands, stencils[n], f, torch.empty_like(f), ax))
        stream = torch.cuda.current_stream()
        tuned = None
        if tune:
            from paper_2101_02286_amd import tune as tuner
            t0 = time.perf_counter()
            item_plans, choices, tres = tuner.tune_batch(spec, precision=prec, refine_iters=iters, reps=5,
                                                         max_ctas=batch_ctas, stream=stream)
            tuned = dict(tres, choices=choices, tune_wall_s=round(time.perf_counter() - t0, 1))
        else:  # one automatic plan per line length
            by_n = {}
            item_plans = []
            for b_, st, f, o, ax in spec:
                n = f.shape[2 - ax]
                if n not in by_n:
                    by_n[n] = cb.Plan(bands, n, precision=prec, refine_iters=iters)
                item_plans.append(by_n[n])
        items = [(pl, st, f, o, ax) for pl, (_b, st, f, o, ax) in zip(item_plans, spec)]
        batch = cb.Batch(items, stream=stream)
        launch = lambda: batch.launch(batch_ctas, stream)
        dur, wall = _time_launches(launch, steps, warmup, stream)
        dof = sum(f.numel() for f in fields) * 3
        ms = float(np.median(dur))
        r = {"ms": round(ms, 4), "gdofs": round(dof / (ms * 1e-3) / 1e9, 2),
             "hbm_gbs_algorithmic": round(16 * dof / (ms * 1e-3) / 1e9, 1), "items": len(items),
             "refine_iters": sorted({pl.info()["refine_iters"] for pl in item_plans}),
             "outputs": [it[3] for it in items]}
        if tuned is not None:
            tuned["automatic_gdofs"] = round(dof / (tuned["automatic_ms"] * 1e-3) / 1e9, 2)
            tuned["automatic_ms"] = round(tuned["automatic_ms"], 4)
            tuned["tuned_ms"] = round(tuned["tuned_ms"], 4)
            r["autotuned"] = tuned
        if extras:
            # the persistent work-queue form of the same launches
            qdur, _ = _time_launches(lambda: batch.launch(0, stream), steps, warmup, stream)
            r["persistent_queue_gdofs"] = round(dof / (float(np.median(qdur)) * 1e-3) / 1e9, 2)
            # the same launches captured once in a HIP graph and replayed
            gs = torch.cuda.Stream()
            gs.wait_stream(stream)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=gs):
                batch.launch(batch_ctas, gs)
            torch.cuda.synchronize()
            gdur, _ = _time_launches(g.replay, steps, warmup, torch.cuda.current_stream())
            gms = float(np.median(gdur))
            r["graph_replay_ms"] = round(gms, 4)
            r["graph_replay_gdofs"] = round(dof / (gms * 1e-3) / 1e9, 2)
        out[key] = r
        torch.cuda.synchronize()
        del batch
        for pl in {id(p_): p_ for p_ in item_plans}.values():
            pl.close()
    # accuracy of the FP32+refinement outputs against the FP64 outputs
    o64s = out["fp64"].pop("outputs")
    for key in out:
        if key == "fp64":
            continue
        worst = 0.0
        for o64, o32 in zip(o64s, out[key].pop("outputs")):
            worst = max(worst, float(((o64 - o32).abs().max() / o64.abs().max()).item()))
        out[key]["max_rel_diff_vs_fp64"] = worst
    return out, shapes


def mode_batched(args):
    """12 uneven periodic grids x 3 axes in one batched launch per kernel class (one workgroup per
    tile; the persistent work-queue form is timed beside it): FP32+refinement vs FP64."""
    # FP64, then FP32 with the library's refinement count (the fewest
    # iterations that reach 1e-12 by its condition-number rule: one for this
    # scheme) and with two (the FP64 floor)
    out, shapes = batched_runs((("fp64", "fp64", 0), ("fp32_refine", "fp32_refine", 0),
                                ("fp32_refine2", "fp32_refine", 2)), args.steps, args.warmup, args.batch_ctas,
                               args.tune)
    return {"metric": "GDOF/s, 12 uneven grids x 3 axes in one batched launch per kernel class", "fp64": out["fp64"],
            "fp32_refine": out["fp32_refine"], "fp32_refine2": out["fp32_refine2"],
            "config": {"workload": "grids %s" % shapes, "autotuned": bool(args.tune)}}


def leg_batched(steps, warmup):
    """The 12-grid batch with plans tuned for the whole batch (the automatic plans' time beside)."""
    out, shapes = batched_runs((("fp64", "fp64", 0), ("fp32_refine", "fp32_refine", 0)), steps, warmup,
                               tune=True, extras=False)
    return {"workload": "12 uneven periodic grids %s x 3 axes, sixth-order derivative, one workgroup per tile, "
                        "plans autotuned for the whole batch" % [list(map(int, s)) for s in shapes],
            "fp64": out["fp64"], "fp32_refine": out["fp32_refine"]}


def serve_run(rate, precision, count, max_points, budget_gb=0.0, seed=11):
    """One served Poisson stream, timed after an untimed pass of the same requests (arriving all at
    once) on the same executor, as in a server that has been running: kernels loaded, the stream
    slots' workspaces and pinned staging buffers made, the device memory pool holding blocks of the
    requests' sizes.  Inputs are staged in HBM and plans factorised before each pass."""
    from paper_2101_02286_amd.serve import GpuExecutor, Server, poisson_requests
    ex = GpuExecutor(slots=8, precision=precision)
    budget = budget_gb * (1 << 30) if budget_gb else None
    for timed in (False, True):
        reqs = poisson_requests(count, rate_hz=rate if timed else 1e9, seed=seed, max_points=max_points)
        ex.stage(reqs)
        st = Server(ex, hbm_budget=budget, slots=8, max_batch=4).run(reqs)
    st["rate_hz"] = rate
    st["precision"] = precision
    del ex
    torch.cuda.empty_cache()
    return st


def leg_served(count, max_points):
    """The served stream at a moderate Poisson rate and all at once (saturation), FP32 + refinement
    and plain FP64 on the same requests."""
    res = {}
    for rate in (400.0, 1e9):
        for prec in ("fp32_refine", "fp64"):
            st = serve_run(rate, prec, count, max_points)
            res["%s@%s" % (prec, "all_at_once" if rate >= 1e9 else "%gHz" % rate)] = {
                k: (round(v, 3) if isinstance(v, float) else v)
                for k, v in st.items() if k in ("requests", "p50_ms", "p99_ms", "gdofs", "span_s",
                                                 "max_inflight_batches", "batches", "max_batch_requests")}
    return {"workload": "%d requests, sides log-uniform [32,1024], <= %.2g points, random axis, tri6/penta10"
                        % (count, max_points), "runs": res}


def mode_serve(args):
    """Poisson request stream served with continuous batching (FP32+refinement)."""
    # 8 stream slots and at most 4 requests per batched launch: small batches
    # keep the slots balanced (measured: saturation p50 11.6 ms vs 21 ms with
    # 4 slots x 16 requests)
    res = [serve_run(rate, "fp32_refine", args.requests, args.max_points, args.budget_gb) for rate in args.rates]
    fp64 = [serve_run(rate, "fp64", args.requests, args.max_points, args.budget_gb) for rate in args.rates]
    return {"metric": "served p50/p99 latency and GDOF/s", "runs": res, "runs_fp64": fp64,
            "saturation_gdofs": round(max(r["gdofs"] for r in res), 2),
            "saturation_gdofs_fp64": round(max(r["gdofs"] for r in fp64), 2),
            "config": {"workload": "Poisson stream, sides log-uniform [32,1024], <= %.2g points, "
                                   "tri6/penta10, FP32+refinement (automatic count: 1 tri6, 2 penta10) and FP64 "
                                   "at the same rates" % args.max_points}}


def mode_copy(args):
    """Plain device copy of a known size (reference for the HBM byte counters)."""
    dev = torch.device("cuda:0")
    a = torch.ones(args.copy_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    dur, wall = _time_launches(lambda: b.copy_(a), args.steps, args.warmup, stream)
    ms = float(dur.mean())
    return {"metric": "device copy", "bytes_read": a.numel() * 8, "bytes_written": a.numel() * 8,
            "ms": round(ms, 4), "gbs": round(2 * a.numel() * 8 / (ms * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="headline",
                    choices=["headline", "two_level", "penta_z", "batched", "serve", "copy"])
    ap.add_argument("--rates", type=float, nargs="+", default=[50.0, 200.0, 800.0, 3200.0, 1e9],
                    help="Poisson arrival rates (requests/s); a huge rate = all requests at once (saturation)")
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--batch-ctas", type=int, default=-1,
                    help="batched launches: < 0 one workgroup per tile (default); 0 persistent queue with all "
                         "workgroups that fit; > 0 persistent queue with at most that many")
    ap.add_argument("--max-points", type=float, default=1.5e8)
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="serving admission budget; 0 = a share of the device's free memory")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only (skip the summaries of the other workloads)")
    ap.add_argument("--serve-requests", type=int, default=240,
                    help="requests per served run in the default (headline) line")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--tune", action="store_true",
                    help="autotune first: the launch shape per direction (headline), the whole batch (batched)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the split across GPUs is designed, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    fn = {"headline": headline, "two_level": mode_two_level, "penta_z": mode_penta_z, "batched": mode_batched,
          "serve": mode_serve, "copy": mode_copy}[args.mode]
    res = fn(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
