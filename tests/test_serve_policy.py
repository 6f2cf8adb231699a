"""CPU tests of the serving policy with a fake clock and a fake executor."""
import pytest

from paper_2101_02286_amd.serve import Request, Server, poisson_requests


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a batch after a duration proportional to its unknowns."""

    def __init__(self, clock, dof_per_s=1e9, overhead=1e-4):
        self.clock, self.rate, self.overhead = clock, dof_per_s, overhead
        self.launches = []
        self.alloc_order = []

    def group_key(self, r):
        return r.scheme

    def alloc(self, r):
        self.alloc_order.append(r.rid)

    def launch(self, slot, reqs):
        t_end = self.clock() + self.overhead + sum(r.dof for r in reqs) / self.rate
        self.launches.append((self.clock(), t_end, slot, [r.rid for r in reqs]))
        return t_end

    def done(self, h):
        return self.clock() >= h

    def release(self, r):
        pass


def run(reqs, budget, slots=3, max_batch=8, step=1e-4):
    clk = Clock()
    ex = FakeExecutor(clk)
    srv = Server(ex, budget, slots=slots, max_batch=max_batch, clock=clk)

    def tick():
        clk.t += step

    st = srv.run(reqs, sleep=tick)
    return srv, ex, st


def test_every_request_completes_within_budget():
    reqs = poisson_requests(60, rate_hz=2000, seed=1, side_lo=16, side_hi=128)
    budget = 4 * max(r.mem for r in reqs)
    srv, ex, st = run(reqs, budget)
    assert st["requests"] == 60
    assert srv.peak_used <= budget
    for r in srv.finished:
        assert r.arrival <= r.admit_t <= r.launch_t <= r.done_t


def test_fifo_admission_no_overtaking():
    big = Request(0, (64, 64, 64), 0, "tri6", 0.0)
    small = [Request(i, (8, 8, 8), 0, "tri6", 1e-6 * i) for i in range(1, 6)]
    budget = big.mem + small[0].mem  # the big one plus at most one small at a time
    srv, ex, st = run([big] + small, budget)
    assert ex.alloc_order == list(range(6))


def test_continuous_batching_overlaps_batches():
    """Requests arriving while a batch runs start on another slot before it ends."""
    reqs = [Request(i, (64, 64, 64), i % 3, "tri6", 2e-5 * i) for i in range(12)]
    srv, ex, st = run(reqs, budget=1 << 40, slots=3)
    assert st["max_inflight_batches"] >= 2
    spans = [(a, b) for a, b, _, _ in ex.launches]
    overlapping = any(spans[i][0] < spans[j][1] and spans[j][0] < spans[i][1]
                      for i in range(len(spans)) for j in range(i + 1, len(spans)))
    assert overlapping


def test_batches_respect_group_and_size():
    reqs = poisson_requests(40, rate_hz=1e6, seed=3, side_lo=8, side_hi=32)
    srv, ex, st = run(reqs, budget=1 << 40, slots=2, max_batch=5)
    byid = {r.rid: r for r in reqs}
    for _, _, _, ids in ex.launches:
        assert 1 <= len(ids) <= 5
        assert len({byid[i].scheme for i in ids}) == 1


def test_oversized_request_rejected():
    clk = Clock()
    srv = Server(FakeExecutor(clk), hbm_budget=1000, clock=clk)
    with pytest.raises(ValueError):
        srv.submit(Request(0, (100, 100, 100), 0, "tri6", 0.0))


def test_poisson_stream_is_seeded_and_bounded():
    a = poisson_requests(50, 100.0, seed=9)
    b = poisson_requests(50, 100.0, seed=9)
    assert [(r.shape, r.axis, r.scheme, r.arrival) for r in a] == [(r.shape, r.axis, r.scheme, r.arrival) for r in b]
    for r in a:
        assert all(32 <= s <= 1024 for s in r.shape)
        assert r.dof <= 1.5e8
