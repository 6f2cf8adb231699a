"""Continuous-batching request server for compact derivative / solve requests.

Requests (a 3D periodic grid, an axis, a scheme) arrive over time.  The
server keeps factorised plans on the device (one per scheme and line length),
admits arrived requests in FIFO order while their device memory fits the HBM
budget, and launches every group of admitted-but-not-started requests as ONE
batched launch (cb_solve_batched: one kernel per kernel class) on a free stream slot -- while
earlier batches are still running on other slots.  Finished batches release
their memory at once, so waiting requests are admitted as slots and memory
free up.  Latency = completion - arrival.

The scheduling policy (`Server`) is independent of the device: it drives an
executor with four calls (alloc, launch, done, release).  `GpuExecutor` runs
the HIP library; tests drive the policy with a fake executor and clock.

Request inputs are staged on the device before the served clock starts
(`GpuExecutor.stage`, standing in for data that a client has already placed
in HBM); admission then accounts for each request's input and output bytes
against a budget taken from the device's free memory (hipMemGetInfo) unless
one is given.
"""
import collections
import math
import time

import numpy as np

from . import schemes


class Request:
    __slots__ = ("rid", "shape", "axis", "scheme", "arrival", "seed", "admit_t", "launch_t", "done_t", "mem",
                 "bufs", "batch")

    def __init__(self, rid, shape, axis, scheme, arrival, seed=0):
        self.rid, self.shape, self.axis, self.scheme = rid, tuple(shape), axis, scheme
        self.arrival, self.seed = arrival, seed
        self.admit_t = self.launch_t = self.done_t = None
        self.mem = 2 * 8 * int(np.prod(self.shape))  # FP64 input + output
        self.bufs = None
        self.batch = None

    @property
    def dof(self):
        return int(np.prod(self.shape))

    @property
    def n(self):
        return self.shape[self.axis]  # shape is (nx, ny, nz)


class Server:
    # defaults: 8 slots and batches of at most 4 requests balanced the slots
    # best on a saturated stream of random-size requests (MI355X)
    def __init__(self, executor, hbm_budget=None, slots=8, max_batch=4, clock=time.perf_counter):
        self.ex = executor
        # no budget given: what the executor reports as free device memory
        self.budget = int(hbm_budget if hbm_budget is not None else executor.budget_bytes())
        self.slots = slots
        self.max_batch = max_batch
        self.clock = clock
        self.pending = collections.deque()   # arrived, not admitted
        self.ready = collections.deque()     # admitted, not launched
        self.inflight = []                   # (slot, handle, [requests])
        self.free_slots = list(range(slots))
        self.used = 0
        self.finished = []
        self.peak_used = 0
        self.max_inflight = 0
        self.batch_sizes = []                # requests per launched batch

    def submit(self, req):
        if req.mem > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.rid, req.mem))
        self.pending.append(req)

    def _retire(self):
        still = []
        for slot, h, reqs in self.inflight:
            if self.ex.done(h):
                t = self.clock()
                for r in reqs:
                    r.done_t = t
                    self.ex.release(r)
                    self.used -= r.mem
                    self.finished.append(r)
                self.free_slots.append(slot)
            else:
                still.append((slot, h, reqs))
        self.inflight = still

    def _admit(self):
        while self.pending and self.used + self.pending[0].mem <= self.budget:
            r = self.pending.popleft()
            self.ex.alloc(r)
            self.used += r.mem
            r.admit_t = self.clock()
            self.ready.append(r)
        self.peak_used = max(self.peak_used, self.used)

    def _launch(self):
        while self.ready and self.free_slots:
            groups = collections.OrderedDict()
            for r in self.ready:
                groups.setdefault(self.ex.group_key(r), []).append(r)
            key, reqs = next(iter(groups.items()))
            reqs = reqs[:self.max_batch]
            for r in reqs:
                self.ready.remove(r)
            slot = self.free_slots.pop(0)
            t = self.clock()
            for r in reqs:
                r.launch_t = t
            h = self.ex.launch(slot, reqs)
            self.batch_sizes.append(len(reqs))
            self.inflight.append((slot, h, reqs))
            self.max_inflight = max(self.max_inflight, len(self.inflight))

    def poll(self):
        """One scheduling round: retire, admit, launch."""
        self._retire()
        self._admit()
        self._launch()

    def idle(self):
        return not (self.pending or self.ready or self.inflight)

    def run(self, requests, sleep=None):
        """Replay requests whose .arrival is relative to the start; returns stats."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        t0 = self.clock()
        for r in reqs:
            r.arrival += t0
        i = 0
        while i < len(reqs) or not self.idle():
            now = self.clock()
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i])
                i += 1
            self.poll()
            if sleep:
                sleep()
        return self.stats(t0)

    def stats(self, t0):
        lat = np.array([r.done_t - r.arrival for r in self.finished])
        span = max(r.done_t for r in self.finished) - t0
        dof = sum(r.dof for r in self.finished)
        return {"requests": len(self.finished), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "gdofs": dof / span / 1e9, "span_s": span, "peak_bytes": self.peak_used,
                "budget_bytes": self.budget, "max_inflight_batches": self.max_inflight,
                "batches": len(self.batch_sizes), "max_batch_requests": max(self.batch_sizes, default=0)}


def poisson_requests(count, rate_hz, seed=0, side_lo=32, side_hi=1024, max_points=1.5e8,
                     schemes=("tri6", "penta10")):
    """Seeded request stream: Poisson arrivals, sides log-uniform in [lo, hi]
    with the product capped, uniform axis and scheme."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate_hz)
        while True:
            sides = np.exp(rng.uniform(math.log(side_lo), math.log(side_hi), size=3))
            sides = [int(round(s)) for s in sides]
            if np.prod(sides, dtype=np.float64) <= max_points:
                break
        out.append(Request(rid, sides, int(rng.integers(0, 3)), schemes[int(rng.integers(0, len(schemes)))],
                           t, seed=int(rng.integers(0, 2 ** 31))))
    return out


class GpuExecutor:
    """Runs request groups as one batched launch per stream slot.

    `precision` defaults to FP64: each line is read and written once either
    way, and FP32 with FP64 refinement runs the reduction at least twice per
    line with both precisions' state in registers, which costs more than
    FP64 arithmetic saves (measured at saturation on the served request
    mix: 170-173 GDOF/s FP64, 89-93 FP32 + refinement); "fp32_refine"
    remains available."""

    # share of the device's free memory that admission may hand to requests
    BUDGET_FRACTION = 0.8

    def __init__(self, slots=8, precision="fp64", refine_iters=0, rows_per_lane=0, device="cuda:0",
                 on_result=None):
        import torch
        from . import cb
        self.torch, self.cb = torch, cb
        self.on_result = on_result  # called as on_result(request, input, output) before release
        self.device = torch.device(device)
        self.precision, self.refine_iters, self.rpl = precision, refine_iters, rows_per_lane
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.ws = {}
        self.plans = {}
        self.stencils = {}
        self.inputs = {}

    def plan(self, scheme, n):
        key = (scheme, n)
        if key not in self.plans:
            self.plans[key] = self.cb.Plan(schemes.bands(scheme), n, precision=self.precision,
                                           refine_iters=self.refine_iters, rows_per_lane=self.rpl)
            self.stencils[key] = self.cb.Stencil(*schemes.stencil(scheme, n))
        return self.plans[key], self.stencils[key]

    def group_key(self, r):
        # a batched launch takes any mix of plans (one kernel launch per
        # kernel class), so every request may join every batch
        return 0

    def stage(self, requests):
        """Place every request's input in HBM (seeded U(0, 1) fields) and
        factorise its plan, before the served clock starts."""
        torch = self.torch
        for r in requests:
            self.plan(r.scheme, r.n)
            if r.rid not in self.inputs:
                nx, ny, nz = r.shape
                g = torch.Generator(device=self.device)
                g.manual_seed(r.seed)
                self.inputs[r.rid] = torch.rand((nz, ny, nx), generator=g, device=self.device, dtype=torch.float64)
        torch.cuda.synchronize(self.device)

    def budget_bytes(self):
        """Admission budget: a share of the device memory free now (hipMemGetInfo)."""
        free, _total = self.torch.cuda.mem_get_info(self.device)
        return int(free * self.BUDGET_FRACTION)

    def alloc(self, r):
        f = self.inputs.get(r.rid)
        if f is None:
            raise KeyError("request %d was not staged" % r.rid)
        r.bufs = (f, self.torch.empty_like(f))

    def launch(self, slot, reqs):
        torch, cb = self.torch, self.cb
        s = self.streams[slot]
        s.wait_stream(torch.cuda.current_stream(self.device))  # inputs written on the current stream
        items = (cb.BatchItem * len(reqs))()
        keep = []
        for i, r in enumerate(reqs):
            plan, st = self.plan(r.scheme, r.n)
            f, out = r.bufs
            items[i].plan = plan.h
            items[i].stencil = cb.ctypes.pointer(st.c)
            items[i].grid = cb.grid_of(f)
            items[i].axis = r.axis
            items[i].inp = f.data_ptr()
            items[i].out = out.data_ptr()
            keep.append(st)
        need = cb.lib().cb_batch_workspace_bytes(items, len(reqs))
        ws = self.ws.get(slot)
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 1 << 16), dtype=torch.uint8, device=self.device)
            self.ws[slot] = ws
        # one workgroup per tile (measured faster than the persistent queue)
        cb._check(cb.lib().cb_solve_batched(items, len(reqs), cb.ctypes.c_void_p(ws.data_ptr()), ws.numel(), -1,
                                            cb.ctypes.c_void_p(s.cuda_stream)))
        ev = torch.cuda.Event()
        ev.record(s)
        for r in reqs:
            r.batch = slot
        return ev

    def done(self, h):
        return h.query()

    def release(self, r):
        if self.on_result is not None:
            self.on_result(r, r.bufs[0], r.bufs[1])
        r.bufs = None
        self.inputs.pop(r.rid, None)

