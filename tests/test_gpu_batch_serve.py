"""GPU tests of the batched persistent launch, its graph replay, and the
continuous-batching server (each result alone equals the result in the mix)."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import schemes
from paper_2101_02286_amd import cb, synth
from paper_2101_02286_amd.serve import GpuExecutor, Server, poisson_requests

pytestmark = pytest.mark.gpu

TRI = schemes.bands_collocated(schemes.DERIV6)
PENTA = schemes.bands_collocated(schemes.DERIV10)
HEPT = schemes.bands_collocated(schemes.DERIV12H)


def relerr(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def stencil_for(scheme, n):
    s = dict(tri6=schemes.DERIV6, penta10=schemes.DERIV10, hept12=schemes.DERIV12H)[scheme]
    lo, c = schemes.stencil_deriv_collocated(s, 2 * math.pi / n)
    return lo, c


def batch(items, stream=None):
    arr = (cb.BatchItem * len(items))()
    keep = []
    for i, (plan, st, f, out, axis) in enumerate(items):
        arr[i].plan = plan.h
        arr[i].stencil = cb.ctypes.pointer(st.c) if st is not None else None
        arr[i].grid = cb.grid_of(f)
        arr[i].axis = axis
        arr[i].inp = f.data_ptr()
        arr[i].out = out.data_ptr()
        keep.append(st)
    need = cb.lib().cb_batch_workspace_bytes(arr, len(items))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s = stream or torch.cuda.current_stream()
    cb._check(cb.lib().cb_batch_build(arr, len(items), cb.ctypes.c_void_p(ws.data_ptr()), need,
                                      cb.ctypes.c_void_p(s.cuda_stream)))
    return ws


def launch(ws, stream=None, max_ctas=0):
    s = stream or torch.cuda.current_stream()
    cb._check(cb.lib().cb_batch_launch(cb.ctypes.c_void_p(ws.data_ptr()), max_ctas,
                                       cb.ctypes.c_void_p(s.cuda_stream)))


@pytest.mark.parametrize("max_ctas", [7, -1])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_uneven_grids_one_launch(gpu, precision, max_ctas):
    """Persistent queue with few workgroups (each loops over many tiles), and
    one workgroup per tile in XCD-grouped order."""
    shapes = [(16, 16, 16), (32, 24, 40), (48, 48, 48), (96, 32, 16), (24, 128, 8), (64, 20, 36)]
    items, refs = [], []
    for gi, (nx, ny, nz) in enumerate(shapes):
        f, _ = synth.random_modes((nz, ny, nx), seed=gi)
        fd = f.to(gpu)
        for axis in range(3):
            n = (nx, ny, nz)[axis]
            lo, c = stencil_for("tri6", n)
            plan = cb.Plan(TRI, n, precision=precision, rows_per_lane=8)
            out = torch.empty_like(fd)
            items.append((plan, cb.Stencil(lo, c), fd, out, axis))
            refs.append(oracle.apply_axis(f.numpy(), axis, TRI, lo, c))
    ws = batch(items)
    launch(ws, max_ctas=max_ctas)
    torch.cuda.synchronize()
    for (plan, st, fd, out, axis), ref in zip(items, refs):
        assert relerr(out.cpu().numpy(), ref) <= 1e-12


def test_batched_solve_items_and_penta(gpu):
    items, refs = [], []
    for i, n in enumerate((37, 100, 256, 613)):
        b = synth.random_uniform((5, 3, n), seed=i).to(gpu)
        plan = cb.Plan(PENTA, n, rows_per_lane=16)
        out = torch.empty_like(b)
        items.append((plan, None, b, out, 0))
        refs.append(oracle.solve_axis(b.cpu().numpy(), 0, PENTA))
    launch(batch(items))
    torch.cuda.synchronize()
    for it, ref in zip(items, refs):
        assert relerr(it[3].cpu().numpy(), ref) <= 1e-12


def test_mixed_plans_one_batch(gpu):
    """Items of different schemes, precisions, lane layouts (uniform, ragged,
    eliminated interiors) and axes in one batch: each matches the oracle and is
    bitwise equal to the same item computed by a single call."""
    cases = [  # (bands, n, precision, refine, per_row, axis, fused, cyclic)
        (TRI, 64, "fp64", 0, False, 0, True, True), (TRI, 96, "fp64", 0, False, 1, True, True),
        (PENTA, 128, "fp32_refine", 3, False, 2, True, True), (TRI, 613, "fp64", 0, False, 0, False, True),
        (PENTA, 384, "fp64", 0, False, 1, False, True), (TRI, 256, "fp32_refine", 2, False, 2, False, True),
        (TRI, 200, "fp64", 0, True, 0, False, True), (PENTA, 512, "fp64", 0, False, 0, True, True),
        (TRI, 256, "fp64", 0, False, 2, True, True), (PENTA, 512, "fp64", 0, False, 1, False, True),
        # acyclic items with the same bands on every row (FP64 and FP32 + refinement)
        (TRI, 300, "fp32_refine", 0, False, 1, False, False), (PENTA, 512, "fp32_refine", 2, False, 0, False, False),
        (TRI, 96, "fp64", 0, False, 2, False, False),
        # heptadiagonal (r = 3) items: fused, FP32 + refinement, acyclic
        (HEPT, 256, "fp64", 0, False, 0, True, True), (HEPT, 300, "fp32_refine", 0, False, 2, False, True),
        (HEPT, 613, "fp64", 0, False, 1, False, False),
    ]
    items, singles, refs = [], [], []
    rng = np.random.default_rng(5)
    for k, (bands, n, prec, it, per_row, axis, fused, cyclic) in enumerate(cases):
        shape = [7, 5]
        shape.insert(axis, n)
        shape = (shape[2], shape[1], shape[0])
        if per_row:
            bd = np.tile(np.asarray(bands, dtype=np.float64), (n, 1))
            bd[:, 1] += rng.uniform(0.0, 0.5, n)  # stays diagonally dominant
            plan = cb.Plan(bd, n, per_row=True, precision=prec, refine_iters=it)
        else:
            bd = bands
            plan = cb.Plan(bands, n, precision=prec, refine_iters=it, cyclic=cyclic)
        if fused:
            f, _ = synth.random_modes(shape, seed=k)
            lo, c = stencil_for("tri6" if bands is TRI else ("penta10" if bands is PENTA else "hept12"), n)
            st = cb.Stencil(lo, c)
            refs.append(oracle.apply_axis(f.numpy(), axis, bands, lo, c))
            fd = f.to(gpu)
            singles.append(cb.apply_derivative(plan, st, fd, axis))
        else:
            b = synth.random_uniform(shape, seed=k)
            st = None
            refs.append(oracle.solve_axis(b.numpy(), axis, bd, per_row=per_row, cyclic=plan.cyclic))
            fd = b.to(gpu)
            singles.append(cb.solve(plan, fd, axis))
        items.append((plan, st, fd, torch.empty_like(fd), axis))
    ws = batch(items)
    for max_ctas in (11, -1):  # persistent queue, then one workgroup per tile
        for it in items:
            it[3].fill_(float("nan"))
        launch(ws, max_ctas=max_ctas)
        torch.cuda.synchronize()
        for (plan, st, fd, out, axis), single, ref in zip(items, singles, refs):
            got = out.cpu().numpy()
            assert relerr(got, ref) <= 1e-12
            assert np.array_equal(got, single.cpu().numpy())


def _partitioned_batch_items(gpu):
    """Items split over workgroup partitions (FP64 and FP32 + refinement,
    fused and plain, cyclic and acyclic, r = 1..3) beside one-partition ones,
    and one-partition plans whose strided launches run a partitioned copy
    (P = 0 below: a ragged 1100-row line and an 8192-row one)."""
    HEPT = schemes.bands_collocated(schemes.DERIV12H)
    cases = [  # (bands, scheme, n, P, precision, axis, fused, cyclic)
        (TRI, "tri6", 4096, 4, "fp64", 0, True, True), (PENTA, "penta10", 3003, 3, "fp32_refine", 2, True, True),
        (TRI, "tri6", 2000, 5, "fp64", 1, False, False), (HEPT, "hept12", 2048, 4, "fp32_refine", 0, False, True),
        (TRI, "tri6", 256, 1, "fp64", 1, True, True), (PENTA, "penta10", 300, 1, "fp32_refine", 0, False, True),
        (TRI, "tri6", 1100, 0, "fp64", 1, True, True), (PENTA, "penta10", 8192, 0, "fp64", 2, False, True),
    ]
    items, singles, refs = [], [], []
    for k, (bands, scheme, n, P, prec, axis, fused, cyclic) in enumerate(cases):
        shape = [6, 5]
        shape.insert(axis, n)
        shape = (shape[2], shape[1], shape[0])
        plan = cb.Plan(bands, n, partitions=P, precision=prec, cyclic=cyclic)
        assert plan.info()["partitions"] == max(P, 1)
        if P == 0:
            assert plan.info()["partitions_strided"] > 1 and axis > 0
        if fused:
            f, _ = synth.random_modes(shape, seed=k)
            lo, c = stencil_for(scheme, n)
            st = cb.Stencil(lo, c)
            refs.append(oracle.apply_axis(f.numpy(), axis, bands, lo, c))
            fd = f.to(gpu)
            singles.append(cb.apply_derivative(plan, st, fd, axis))
        else:
            b = synth.random_uniform(shape, seed=k)
            st = None
            refs.append(oracle.solve_axis(b.numpy(), axis, bands, cyclic=cyclic))
            fd = b.to(gpu)
            singles.append(cb.solve(plan, fd, axis))
        items.append((plan, st, fd, torch.empty_like(fd), axis))
    return items, singles, refs


def test_batch_with_partitioned_items(gpu):
    """P > 1 items run as their own phase launches after the line classes,
    with their scratch in the workspace: each matches the oracle and is
    bitwise equal to its single call."""
    items, singles, refs = _partitioned_batch_items(gpu)
    ws = batch(items)
    assert ws.numel() > cb.lib().cb_batch_workspace_size(len(items))
    for max_ctas in (5, -1):
        for it in items:
            it[3].fill_(float("nan"))
        launch(ws, max_ctas=max_ctas)
        torch.cuda.synchronize()
        for (plan, st, fd, out, axis), single, ref in zip(items, singles, refs):
            got = out.cpu().numpy()
            assert relerr(got, ref) <= 1e-12
            assert np.array_equal(got, single.cpu().numpy())


def test_graph_replay_with_partitioned_items(gpu):
    """The batched launch with P > 1 items captured once in a HIP graph and
    replayed several times, with eager work between the replays: every
    replay equals the eager result."""
    items, singles, refs = _partitioned_batch_items(gpu)
    ws = batch(items)
    torch.cuda.synchronize()
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=gs):
        launch(ws, stream=gs, max_ctas=-1)
    torch.cuda.synchronize()
    for rep in range(3):
        for it in items:
            it[3].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device=gpu).sum()  # eager work between replays
        torch.cuda.synchronize()
        for (plan, st, fd, out, axis), single in zip(items, singles):
            assert torch.equal(out, single), rep
    del junk


def test_batch_with_empty_items(gpu):
    """Items with no lines (first, middle, last) take no tiles; the others are solved."""
    plan = cb.Plan(TRI, 64, rows_per_lane=8)
    items, refs = [], []
    for k, shape in enumerate(((0, 3, 64), (4, 3, 64), (2, 0, 64), (3, 5, 64), (0, 0, 64))):
        b = synth.random_uniform(shape, seed=k).to(gpu)
        out = torch.full_like(b, 7.0)
        items.append((plan, None, b, out, 0))
        refs.append(oracle.solve_axis(b.cpu().numpy(), 0, TRI) if b.numel() else None)
    launch(batch(items), max_ctas=3)
    torch.cuda.synchronize()
    for it, ref in zip(items, refs):
        if ref is not None:
            assert relerr(it[3].cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("max_ctas", [0, -1])
def test_graph_replay_of_batched_launch(gpu, max_ctas):
    """Captured launch replayed several times with eager work in between."""
    f, _ = synth.random_modes((24, 40, 32), seed=4)
    fd = f.to(gpu)
    items = []
    for axis in range(3):
        n = fd.shape[2 - axis]
        lo, c = stencil_for("tri6", n)
        items.append((cb.Plan(TRI, n, rows_per_lane=8), cb.Stencil(lo, c), fd, torch.empty_like(fd), axis))
    s = torch.cuda.Stream()
    ws = batch(items, stream=s)
    launch(ws, stream=s, max_ctas=max_ctas)
    s.synchronize()
    eager = [it[3].clone() for it in items]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        launch(ws, stream=s, max_ctas=max_ctas)
    for rep in range(4):
        for it in items:
            it[3].fill_(float(rep))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, e in zip(items, eager):
            assert torch.equal(it[3], e), rep


def test_batch_table_upload_streams(gpu):
    """The work table goes up asynchronously on the build stream: a launch on
    another stream waits for it (on the host while that stream is being
    captured), and a rebuilt workspace carries the new table."""
    f, _ = synth.random_modes((20, 36, 28), seed=9)
    fd = f.to(gpu)
    sets = []
    for scheme, bands in (("tri6", TRI), ("penta10", PENTA)):
        items, refs = [], []
        for axis in range(3):
            n = fd.shape[2 - axis]
            lo, c = stencil_for(scheme, n)
            items.append((cb.Plan(bands, n), cb.Stencil(lo, c), fd, torch.empty_like(fd), axis))
            refs.append(oracle.apply_axis(f.numpy(), axis, bands, lo, c))
        sets.append((items, refs))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ws = None
    for items, refs in sets + sets:  # the second round rebuilds the same workspace
        if ws is None:
            ws = batch(items, stream=sa)
        else:
            arr = (cb.BatchItem * len(items))()
            for i, (plan, st, x, out, axis) in enumerate(items):
                arr[i].plan, arr[i].stencil, arr[i].grid = plan.h, cb.ctypes.pointer(st.c), cb.grid_of(x)
                arr[i].axis, arr[i].inp, arr[i].out = axis, x.data_ptr(), out.data_ptr()
            cb._check(cb.lib().cb_batch_build(arr, len(items), cb.ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                              cb.ctypes.c_void_p(sa.cuda_stream)))
        launch(ws, stream=sb)
        sb.synchronize()
        for it, ref in zip(items, refs):
            assert relerr(it[3].cpu().numpy(), ref) <= 1e-12
            it[3].zero_()
        torch.cuda.synchronize()
    # captured on a third stream after a rebuild on the first
    items, refs = sets[0]
    arr = (cb.BatchItem * len(items))()
    for i, (plan, st, x, out, axis) in enumerate(items):
        arr[i].plan, arr[i].stencil, arr[i].grid = plan.h, cb.ctypes.pointer(st.c), cb.grid_of(x)
        arr[i].axis, arr[i].inp, arr[i].out = axis, x.data_ptr(), out.data_ptr()
    cb._check(cb.lib().cb_batch_build(arr, len(items), cb.ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      cb.ctypes.c_void_p(sa.cuda_stream)))
    sc = torch.cuda.Stream()  # the capture waits for the upload on the host
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=sc):
        launch(ws, stream=sc)
    for rep in range(3):
        for it in items:
            it[3].fill_(float(rep))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, ref in zip(items, refs):
            assert relerr(it[3].cpu().numpy(), ref) <= 1e-12, rep


@pytest.mark.parametrize("precision", ["fp32_refine", "fp64"])
def test_server_results_same_alone_and_in_mix(gpu, precision):
    """Requests drawn from the served stream's distribution (sides
    log-uniform in [32, 1024], at most 1.5e8 points, both schemes, all axes,
    mostly ragged line lengths) all arrive at once, so the server runs them
    as several multi-request batches in flight together.  Each result must be
    bitwise equal to the request run alone, and match the oracle, whose
    stencils come from the pinned scheme table (not the server's)."""
    results = {}

    def keep(r, f, out):
        results[r.rid] = (f.cpu().numpy(), out.cpu().numpy())

    reqs = poisson_requests(6, rate_hz=1e9, seed=8)
    assert {r.scheme for r in reqs} == {"tri6", "penta10"} and {r.axis for r in reqs} == {0, 1, 2}
    ex = GpuExecutor(slots=3, precision=precision, on_result=keep)
    ex.stage(reqs)
    srv = Server(ex, slots=3, max_batch=2)
    st = srv.run(reqs)
    assert st["requests"] == len(reqs)
    assert st["max_batch_requests"] >= 2 and st["max_inflight_batches"] >= 2, st
    for r in reqs:
        f, out_mix = results[r.rid]
        plan, stc = ex.plan(r.scheme, r.n)
        fd = torch.from_numpy(f).to(gpu)
        alone = torch.full_like(fd, float("nan"))
        launch(batch([(plan, stc, fd, alone, r.axis)]))
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), out_mix), r.rid  # bitwise
        bands = TRI if r.scheme == "tri6" else PENTA
        lo, c = stencil_for(r.scheme, r.n)
        ref = oracle.apply_axis(f, r.axis, bands, lo, c)
        assert relerr(out_mix, ref) <= 1e-12, r.rid


@pytest.mark.parametrize("precision,iters", [("fp64", 0), ("fp32_refine", 2), ("fp32_refine", 0)])
def test_uneven_grid_batch_full_size(gpu, precision, iters):
    """The benchmark's batch (12 uneven grids x 3 axes, seeded shapes and
    inputs, one launch per kernel class) at full size; every line of every
    item against the oracle (outputs prefilled with NaN)."""
    shapes = synth.grid_batch_shapes(seed=0, count=12)
    items, plans = [], {}
    for gi, (nx, ny, nz) in enumerate(shapes):
        f, _ = synth.random_modes((nz, ny, nx), seed=gi, device=gpu)
        for axis in range(3):
            n = (nx, ny, nz)[axis]
            if n not in plans:
                lo, c = stencil_for("tri6", n)
                plans[n] = (cb.Plan(TRI, n, precision=precision, refine_iters=iters), cb.Stencil(lo, c), lo, c)
            items.append((plans[n][0], plans[n][1], f, torch.full_like(f, float("nan")), axis))
    launch(batch(items))
    torch.cuda.synchronize()
    for plan, st, f, out, axis in items:
        n = f.shape[2 - axis]
        ref = oracle.apply_axis(f.cpu().numpy(), axis, TRI, plans[n][2], plans[n][3])
        assert relerr(out.cpu().numpy(), ref) <= 1e-12, (tuple(f.shape), axis)
