"""Benchmark: cyclic compact-banded PCR solves on one MI355X.

Default workload (the headline): a 512^3 periodic FP64 grid, sixth-order
compact first derivative (cyclic tridiagonal, alpha = 1/3) fused with its
right-hand-side stencil, along x, y and z.  One step = the three directions
(3 x 134,217,728 solved unknowns).  Inputs are resident in HBM before timing.

Prints ONE JSON line (rank 0).  `value` is GDOF/s (solved unknowns per
second); `roofline` uses the algorithmic 16 bytes per unknown (read f, write
f') of the dominant kernel launch, timed with HIP events on the launch stream.
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

from paper_2101_02286_amd import cb, synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
BYTES_PER_DOF = 16


def tri6():
    # sixth-order collocated compact derivative: bands [1/3, 1, 1/3],
    # RHS a (f_{j+1}-f_{j-1})/(2h) + b (f_{j+2}-f_{j-2})/(4h), a = 14/9, b = 1/9
    return [1 / 3, 1.0, 1 / 3], (14 / 9, 1 / 9)


def deriv_stencil(n, a, b):
    h = 2 * math.pi / n
    return cb.Stencil(-2, [-b / (4 * h), -a / (2 * h), 0.0, a / (2 * h), b / (4 * h)])


def cpu_baseline(f_dev, bands, stencils, max_seconds=30.0):
    """The FP64 oracle on the host cores, over a bounded sample of the same work."""
    import oracle
    f = f_dev.cpu().numpy()
    nz, ny, nx = f.shape
    # sample: a slab of z-planes for x and y, a slab of y-rows for z
    slab = max(1, nz // 8)
    t_total, dof = 0.0, 0
    for axis in range(3):
        st = stencils[axis]
        if axis < 2:
            sub = np.ascontiguousarray(f[:slab])
        else:
            sub = np.ascontiguousarray(f[:, :max(1, ny // 8), :])
        t0 = time.perf_counter()
        oracle.apply_axis(sub, axis, bands, st.lo, st.coefs)
        t_total += time.perf_counter() - t0
        dof += sub.size
        if t_total > max_seconds:
            break
    return {"value": dof / t_total / 1e9, "unit": "GDOF/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle (banded LU + Woodbury, OpenMP over lines) on 1/8 of the 512^3 grid per "
                      "direction (x, y: %d z-planes; z: %d y-rows), %.1f s" % (slab, max(1, ny // 8), t_total)}


def headline(args):
    dev = torch.device("cuda:0")
    n = args.n
    shape = (n, n, n)
    bands, (a, b) = tri6()
    plan = cb.Plan(bands, n)
    st = deriv_stencil(n, a, b)
    f, _ = synth.random_modes(shape, seed=0, device=dev)
    outs = [torch.empty_like(f) for _ in range(3)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        for ax in range(3):
            cb.apply_derivative(plan, st, f, ax, out=outs[ax], stream=stream)
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        for ax in range(3):
            ev[k][ax][0].record(stream)
            cb.apply_derivative(plan, st, f, ax, out=outs[ax], stream=stream)
            ev[k][ax][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dur = np.array([[ev[k][ax][0].elapsed_time(ev[k][ax][1]) for ax in range(3)] for k in range(args.steps)])
    dof = n ** 3
    per_dir_ms = dur.mean(axis=0)
    step_ms = wall * 1e3 / args.steps
    value = 3 * dof / (wall / args.steps) / 1e9
    dom = int(np.argmax(per_dir_ms))
    achieved = BYTES_PER_DOF * dof / (per_dir_ms[dom] * 1e-3) / 1e9
    lat = dur.reshape(-1)
    res = {
        "metric": "GDOF/s (solved unknowns per second), 512^3 cyclic tridiagonal compact derivative x/y/z",
        "value": round(value, 3), "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (8 seeded random Fourier modes, seed 0)",
        "config": {"workload": "%d^3 periodic grid, sixth-order compact first derivative (cyclic tridiagonal "
                               "alpha=1/3) fused with its stencil, along x, y, z" % n,
                   "n": n, "lines_per_direction": n * n, "partitions": 1,
                   "lanes": plan.info()["lanes"], "rows_per_lane": plan.info()["rows_per_lane"]},
        "per_direction_ms": {k: round(float(v), 4) for k, v in zip("xyz", per_dir_ms)},
        "per_direction_gdofs": {k: round(dof / (float(v) * 1e-3) / 1e9, 2) for k, v in zip("xyz", per_dir_ms)},
        "achieved_hbm_gbs_algorithmic": {k: round(BYTES_PER_DOF * dof / (float(v) * 1e-3) / 1e9, 1)
                                         for k, v in zip("xyz", per_dir_ms)},
        "solve_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                             "p99": round(float(np.percentile(lat, 99)), 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_line %s-direction (%s)" % ("xyz"[dom], "unit stride" if dom == 0 else "strided"),
                     "bytes_per_launch": BYTES_PER_DOF * dof},
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(f, bands, [st, st, st], max_seconds=args.cpu_seconds)
    plan.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU only (the multi-GPU split is a design, not part of this build)",
              file=sys.stderr)
        sys.exit(2)
    res = headline(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
