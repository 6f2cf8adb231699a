"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 and FP32+refinement results must match the oracle to a
relative max error of 1e-12 (max |x - x_ref| / max |x_ref|); plain FP32 to
1e-6 where the matrix's condition number allows it (tridiagonal schemes),
else to 2 kappa 2^-24 (fp32_bound).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import schemes
from paper_2101_02286_amd import cb, synth

pytestmark = pytest.mark.gpu

TRI = schemes.bands_collocated(schemes.DERIV6)
PENTA = schemes.bands_collocated(schemes.DERIV10)
INTERP = [float(schemes.INTERP6["alpha"]), 1.0, float(schemes.INTERP6["alpha"])]


def relerr(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def deriv_stencil(scheme, n):
    lo, c = schemes.stencil_deriv_collocated(scheme, 2 * math.pi / n)
    return lo, c


def shape_with(axis, n, other=(12, 20)):
    dims = [other[0], other[1]]
    dims.insert(axis, n)  # dims in (x, y, z) order
    return (dims[2], dims[1], dims[0])


# ---------------------------------------------------------- fused derivative
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c1_32cubed_derivative(gpu, axis):
    shape = (32, 32, 32)
    f, modes = synth.random_modes(shape, seed=0)
    lo, c = deriv_stencil(schemes.DERIV6, 32)
    plan = cb.Plan(TRI, 32)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), axis, TRI, lo, c)
    assert relerr(out, ref) <= 1e-12


STAG = [float(schemes.STAG6["alpha"]), 1.0, float(schemes.STAG6["alpha"])]


@pytest.mark.parametrize("scheme", ["deriv6", "interp6", "deriv10", "interp6_s2c", "stag6_c2s", "stag6_s2c"])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [64, 96, 192, 256])
def test_fused_operators(gpu, scheme, axis, n):
    """Collocated derivatives, collocated<->staggered interpolation and the
    staggered derivative (Eq. (1), (2), App. A.2), fused with their stencils."""
    shape = shape_with(axis, n)
    f, _ = synth.random_modes(shape, seed=n + axis)
    h = 2 * math.pi / n
    if scheme == "interp6":
        bands, (lo, c) = INTERP, schemes.stencil_interp_c2s(schemes.INTERP6)
    elif scheme == "interp6_s2c":
        bands, (lo, c) = INTERP, schemes.stencil_interp_s2c(schemes.INTERP6)
    elif scheme == "stag6_c2s":
        bands, (lo, c) = STAG, schemes.stencil_deriv_c2s(schemes.STAG6, h)
    elif scheme == "stag6_s2c":
        bands, (lo, c) = STAG, schemes.stencil_deriv_s2c(schemes.STAG6, h)
    elif scheme == "deriv6":
        bands, (lo, c) = TRI, deriv_stencil(schemes.DERIV6, n)
    else:
        bands, (lo, c) = PENTA, deriv_stencil(schemes.DERIV10, n)
    plan = cb.Plan(bands, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), axis, bands, lo, c)
    assert relerr(out, ref) <= 1e-12


# ---------------------------------------------------------------- solves ---
@pytest.mark.parametrize("bands", ["tri", "penta"])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [5, 8, 32, 37, 128, 512, 613, 1024])
def test_solve_random_rhs(gpu, bands, axis, n):
    bd = TRI if bands == "tri" else PENTA
    if n < len(bd):  # a cyclic system needs n >= 2r + 1 rows
        pytest.skip("n too small")
    shape = shape_with(axis, n, other=(9, 7))
    b = synth.random_uniform(shape, seed=n * 3 + axis)
    plan = cb.Plan(bd, n)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, bd)
    assert relerr(x, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("bands,n", [(TRI, 512), (TRI, 613), (PENTA, 200), (PENTA, 512), (TRI, 5), (PENTA, 9)])
def test_solve_acyclic_constant_bands(gpu, axis, prec, bands, n):
    """Acyclic systems with the same bands on every row (the first and last r
    rows lose the entries outside the matrix), FP64 and FP32 + refinement,
    whose FP64 residual must use those truncated end rows."""
    shape = shape_with(axis, n, other=(9, 7))
    b = synth.random_uniform(shape, seed=n + 5 * axis)
    plan = cb.Plan(bands, n, cyclic=False, precision=prec)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, bands, cyclic=False)
    assert relerr(x, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_solve_acyclic_and_per_row(gpu, axis):
    n = 200
    shape = shape_with(axis, n, other=(5, 6))
    b = synth.random_uniform(shape, seed=axis)
    bands = synth.random_bands(n, 2, seed=axis)
    for cyclic in (True, False):
        plan = cb.Plan(bands, n, per_row=True, cyclic=cyclic)
        x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
        ref = oracle.solve_axis(b.numpy(), axis, bands, per_row=True, cyclic=cyclic)
        assert relerr(x, ref) <= 1e-12, cyclic


@pytest.mark.parametrize("P", [1, 4])
@pytest.mark.parametrize("bands", ["tri", "penta"])
def test_solve_in_place_and_strided_view(gpu, P, bands):
    """In place on a non-contiguous view (x stride 2), one-partition and
    partitioned lines; rows outside the view stay untouched."""
    n = 128
    bd = TRI if bands == "tri" else PENTA
    big = synth.random_uniform((10, 128, 2 * n), seed=5).to(gpu)
    view = big[:, 3:99, ::2]  # non-contiguous: x stride 2
    b = view.cpu().numpy()
    plan = cb.Plan(bd, n, partitions=P)
    cb.solve(plan, view, 0, out=view)  # in place on a strided view
    ref = oracle.solve_axis(np.ascontiguousarray(b), 0, bd)
    assert relerr(view.cpu().numpy(), ref) <= 1e-12
    # rows outside the view are untouched
    before = synth.random_uniform((10, 128, 2 * n), seed=5).numpy()
    after = big.cpu().numpy()
    mask = np.ones(after.shape, bool)
    mask[:, 3:99, ::2] = False
    assert np.array_equal(after[mask], before[mask])


@pytest.mark.parametrize("P", [2, 3, 5, 16])
@pytest.mark.parametrize("bands", ["tri", "penta"])
@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("xs", [1, 2])
def test_partitioned_lines(gpu, P, bands, axis, xs):
    bd = TRI if bands == "tri" else PENTA
    n = 64 * P + 7
    shape = shape_with(axis, n, other=(6, 5))
    b = synth.random_uniform(shape, seed=P)
    plan = cb.Plan(bd, n, partitions=P, x_staging=xs, lines_per_wg=2 if xs == 1 else 0)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, bd)
    assert relerr(x, ref) <= 1e-12


@pytest.mark.parametrize("P", [3, 4])
@pytest.mark.parametrize("bands", ["tri", "penta"])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_partitioned_acyclic_lines(gpu, P, bands, axis):
    """Acyclic systems split over P workgroup partitions: the first partition
    has no coupling to the last one (no corner blocks)."""
    bd = TRI if bands == "tri" else PENTA
    n = 80 * P + 3
    shape = shape_with(axis, n, other=(6, 5))
    b = synth.random_uniform(shape, seed=10 + P + axis)
    plan = cb.Plan(bd, n, partitions=P, cyclic=False)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, bd, cyclic=False)
    assert relerr(x, ref) <= 1e-12


@pytest.mark.parametrize("n", [4100, 6000, 10000])
def test_long_ragged_unit_stride_lines(gpu, n):
    """Ragged unit-stride lines longer than 4096 rows: 16-row lanes in one
    workgroup while 512 lanes suffice, else the plan's workgroup partitions
    (solve and fused derivative)."""
    shape = (3, 2, n)
    b = synth.random_uniform(shape, seed=n)
    plan = cb.Plan(TRI, n)
    x = cb.solve(plan, b.to(gpu), 0).cpu().numpy()
    assert relerr(x, oracle.solve_axis(b.numpy(), 0, TRI)) <= 1e-12
    f, _ = synth.random_modes(shape, seed=n)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), 0).cpu().numpy()
    assert relerr(out, oracle.apply_axis(f.numpy(), 0, TRI, lo, c)) <= 1e-12


HEPT = schemes.bands_collocated(schemes.DERIV12H)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [7, 96, 256, 300, 613])
@pytest.mark.parametrize("cyclic", [True, False])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_heptadiagonal_solve(gpu, axis, n, cyclic, prec):
    """r = 3 (the general band of Sec. 2 Eq. (4)): the twelfth-order scheme's
    heptadiagonal matrix along every axis, uniform (96, 256) and ragged lines,
    cyclic and acyclic, FP64 and FP32 + refinement (automatic count)."""
    b = synth.random_uniform(shape_with(axis, n, (6, 10)), seed=n + 3 * axis + cyclic)
    plan = cb.Plan(HEPT, n, cyclic=cyclic, precision=prec)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, HEPT, cyclic=cyclic)
    assert relerr(x, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n", [64, 512, 613])
def test_heptadiagonal_fused_derivative(gpu, axis, n):
    """Twelfth-order compact derivative (7-point stencil fused with the
    heptadiagonal solve) against the oracle."""
    f, _ = synth.random_modes(shape_with(axis, n, (5, 6)), seed=n + axis)
    lo, c = deriv_stencil(schemes.DERIV12H, n)
    plan = cb.Plan(HEPT, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), axis, HEPT, lo, c)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("cyclic", [True, False])
def test_heptadiagonal_partitioned(gpu, P, axis, cyclic):
    """r = 3 lines split over P workgroup partitions (solve), and the fused
    derivative on the cyclic ones."""
    n = 128 * P + 5
    b = synth.random_uniform(shape_with(axis, n, (5, 6)), seed=P + axis)
    plan = cb.Plan(HEPT, n, partitions=P, cyclic=cyclic)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    assert relerr(x, oracle.solve_axis(b.numpy(), axis, HEPT, cyclic=cyclic)) <= 1e-12
    if cyclic:
        f, _ = synth.random_modes(shape_with(axis, n, (5, 6)), seed=P)
        lo, c = deriv_stencil(schemes.DERIV12H, n)
        out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
        assert relerr(out, oracle.apply_axis(f.numpy(), axis, HEPT, lo, c)) <= 1e-12


def test_heptadiagonal_long_lines(gpu):
    """n = 8192 heptadiagonal lines: unit-stride whole, strided in workgroup partitions."""
    n = 8192
    plan = cb.Plan(HEPT, n)
    for axis in (0, 2):
        b = synth.random_uniform(shape_with(axis, n, (3, 4)), seed=axis)
        x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
        assert relerr(x, oracle.solve_axis(b.numpy(), axis, HEPT)) <= 1e-12, axis


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("n,prec", [(512, "fp64"), (500, "fp64"), (613, "fp64"), (384, "fp32_refine"), (64, "fp64")])
def test_copy_lines_moves_the_data_unchanged(gpu, axis, n, prec):
    """cb_copy_lines (the solve's launch without arithmetic) writes every
    element of the output with its input value, on every axis and layout."""
    f = synth.random_uniform(shape_with(axis, n, (6, 40)), seed=n + axis).to(gpu)
    plan = cb.Plan(TRI, n, precision=prec)
    out = torch.full_like(f, float("nan"))
    cb.copy_lines(plan, f, axis, out=out)
    torch.cuda.synchronize()
    assert torch.equal(out, f)
    # strided launches of long one-partition lines run in partitions: refused
    if axis > 0:
        plan8 = cb.Plan(TRI, 8192)
        g = torch.zeros(shape_with(axis, 8192, (4, 2)), dtype=torch.float64, device=gpu)
        with pytest.raises(cb.CbError):
            cb.copy_lines(plan8, g, axis, out=torch.empty_like(g))


@pytest.mark.parametrize("P", [4, 7, 16])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bands", ["tri", "penta", "hept"])
def test_partitioned_fp32_refinement(gpu, P, axis, bands):
    """FP32 + FP64 refinement across workgroup partitions: every iteration
    runs the partitioned solve (interiors in FP32) on the FP64 residual.
    Solve (cyclic and acyclic) and fused derivative to 1e-12 with the
    automatic count; plain FP32 to its bound; in place is refused."""
    bd, sch = dict(tri=(TRI, schemes.DERIV6), penta=(PENTA, schemes.DERIV10), hept=(HEPT, schemes.DERIV12H))[bands]
    n = 200 * P + 3
    shape = shape_with(axis, n, (5, 6))
    b = synth.random_uniform(shape, seed=P + 10 * axis)
    bdev = b.to(gpu)
    for cyclic in (True, False):
        plan = cb.Plan(bd, n, partitions=P, precision="fp32_refine", cyclic=cyclic)
        assert plan.info()["refine_iters"] >= 1
        x = cb.solve(plan, bdev, axis).cpu().numpy()
        assert relerr(x, oracle.solve_axis(b.numpy(), axis, bd, cyclic=cyclic)) <= 1e-12, cyclic
        with pytest.raises(cb.CbError):  # in place: b is needed again after x is written
            cb.solve(plan, bdev, axis, out=bdev)
    f, _ = synth.random_modes(shape, seed=P)
    lo, c = deriv_stencil(sch, n)
    ref = oracle.apply_axis(f.numpy(), axis, bd, lo, c)
    plan = cb.Plan(bd, n, partitions=P, precision="fp32_refine")
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    assert relerr(out, ref) <= 1e-12
    plan32 = cb.Plan(bd, n, partitions=P, precision="fp32")
    out32 = cb.apply_derivative(plan32, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    assert relerr(out32, ref) <= fp32_bound(bd)


@pytest.mark.parametrize("axis", [1, 2, 0])
@pytest.mark.parametrize("n,bands,cyclic", [(1100, "tri", True), (3000, "penta", True), (2500, "tri", True),
                                            (2048, "penta", False)])
def test_ragged_mid_length_strided_partitions(gpu, axis, n, bands, cyclic):
    """FP64 lines of 1025..4096 rows on general lane layouts: strided launches
    run in ~512-row workgroup partitions (unit-stride lines stay whole); the
    fused derivative (solve only for the acyclic case) against the oracle."""
    bd = TRI if bands == "tri" else PENTA
    plan = cb.Plan(bd, n, cyclic=cyclic)
    assert plan.info()["partitions_strided"] == (n + 511) // 512
    assert plan.info()["partitions"] == 1
    shape = shape_with(axis, n, (5, 7))
    if cyclic:
        f, _ = synth.random_modes(shape, seed=n + axis)
        lo, c = deriv_stencil(schemes.DERIV6 if bands == "tri" else schemes.DERIV10, n)
        out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
        ref = oracle.apply_axis(f.numpy(), axis, bd, lo, c)
    else:
        b = synth.random_uniform(shape, seed=n + axis)
        out = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
        ref = oracle.solve_axis(b.numpy(), axis, bd, cyclic=False)
    plan.close()
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("axis", [1, 2])
@pytest.mark.parametrize("n,bands", [(2500, "tri"), (8192, "penta"), (3000, "tri")])
def test_fp32_strided_partition_copies(gpu, axis, n, bands):
    """FP32 + refinement one-partition plans whose strided launches run a
    ~512-row partitioned copy (n > 4096, or general layouts above 2048 rows):
    fused derivative and out-of-place solve to 1e-12, and an in-place solve
    (which runs whole lines, as the partitioned refinement re-reads b)."""
    bd = TRI if bands == "tri" else PENTA
    plan = cb.Plan(bd, n, precision="fp32_refine")
    assert plan.info()["partitions"] == 1
    assert plan.info()["partitions_strided"] == (n + 511) // 512
    shape = shape_with(axis, n, (5, 6))
    f, _ = synth.random_modes(shape, seed=n + axis)
    lo, c = deriv_stencil(schemes.DERIV6 if bands == "tri" else schemes.DERIV10, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    assert relerr(out, oracle.apply_axis(f.numpy(), axis, bd, lo, c)) <= 1e-12
    b = synth.random_uniform(shape, seed=n + axis + 1)
    ref = oracle.solve_axis(b.numpy(), axis, bd)
    assert relerr(cb.solve(plan, b.to(gpu), axis).cpu().numpy(), ref) <= 1e-12
    bi = b.to(gpu)
    cb.solve(plan, bi, axis, out=bi)
    assert relerr(bi.cpu().numpy(), ref) <= 1e-12
    plan.close()


@pytest.mark.parametrize("axis", [0, 2])
def test_long_fp32_lines_default_partitions(gpu, axis):
    """FP32 + refinement lines longer than one workgroup (n > 8192) are split
    into ~1024-row partitions by default."""
    n = 12000
    plan = cb.Plan(TRI, n, precision="fp32_refine")
    assert plan.info()["partitions"] == 12
    b = synth.random_uniform(shape_with(axis, n, (3, 4)), seed=axis)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    assert relerr(x, oracle.solve_axis(b.numpy(), axis, TRI)) <= 1e-12


@pytest.mark.parametrize("rows", [256, 512, 1024])
@pytest.mark.parametrize("P", [4, 16])
def test_full_block_fp32_refinement(gpu, rows, P):
    """FP32 (+ FP64 refinement) on unit-stride tridiagonal lines of equal
    partitions: phase C solves each whole partition as one block in FP32,
    and each refinement iteration adds its correction to x in place (the
    interface rows included).  Solve (cyclic and acyclic) and fused
    derivative to 1e-12; plain FP32 to its bound."""
    n = rows * P
    shape = shape_with(0, n, (5, 3))
    b = synth.random_uniform(shape, seed=rows + P)
    for cyclic in (True, False):
        plan = cb.Plan(TRI, n, partitions=P, precision="fp32_refine", cyclic=cyclic)
        assert plan.info()["fullblock_seg"] >= 0
        x = cb.solve(plan, b.to(gpu), 0).cpu().numpy()
        assert relerr(x, oracle.solve_axis(b.numpy(), 0, TRI, cyclic=cyclic)) <= 1e-12, cyclic
    f, _ = synth.random_modes(shape, seed=rows)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    ref = oracle.apply_axis(f.numpy(), 0, TRI, lo, c)
    for prec, tol in (("fp32_refine", 1e-12), ("fp32", fp32_bound(TRI))):
        plan = cb.Plan(TRI, n, partitions=P, precision=prec)
        out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), 0).cpu().numpy()
        assert relerr(out, ref) <= tol, prec


@pytest.mark.parametrize("P", [4, 16])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bands", ["tri", "penta", "hept"])
def test_full_block_phase_c(gpu, P, axis, bands):
    """Equal partitions of L*M rows with constant bands: phase C solves each
    whole partition as one block (interface rows as identity equations, the
    uniform lane code with two couplings masked).  Solve (cyclic and acyclic)
    and fused derivative against the oracle, and against the per-interior
    form (x_staging = 1 keeps it on unit-stride lines)."""
    bd, sch = dict(tri=(TRI, schemes.DERIV6), penta=(PENTA, schemes.DERIV10), hept=(HEPT, schemes.DERIV12H))[bands]
    n = 512 * P
    shape = shape_with(axis, n, (4, 5))
    b = synth.random_uniform(shape, seed=P + axis)
    for cyclic in (True, False):
        plan = cb.Plan(bd, n, partitions=P, cyclic=cyclic)
        info = plan.info()
        assert info["fullblock_seg"] >= 0 and info["fullblock_seg_strided"] >= 0
        x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
        ref = oracle.solve_axis(b.numpy(), axis, bd, cyclic=cyclic)
        assert relerr(x, ref) <= 1e-12, cyclic
        if axis == 0:
            general = cb.Plan(bd, n, partitions=P, cyclic=cyclic, x_staging=1)
            xg = cb.solve(general, b.to(gpu), axis).cpu().numpy()
            assert relerr(xg, ref) <= 1e-12 and relerr(x, xg) <= 1e-12
    f, _ = synth.random_modes(shape, seed=P)
    lo, c = deriv_stencil(sch, n)
    plan = cb.Plan(bd, n, partitions=P)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    assert relerr(out, oracle.apply_axis(f.numpy(), axis, bd, lo, c)) <= 1e-12


@pytest.mark.parametrize("rows", [128, 256, 1024, 2048])
@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("bands", ["tri", "penta"])
def test_full_block_partition_sizes(gpu, rows, axis, bands):
    """Full-block phase C on partitions shorter and longer than 512 rows: its
    tridiagonal lanes load the first block-PCR levels' multipliers with the
    data (levels a short partition lacks are never used, a long one's later
    levels are read in the level loop), on 1-2 lines per workgroup."""
    bd, sch = dict(tri=(TRI, schemes.DERIV6), penta=(PENTA, schemes.DERIV10))[bands]
    P = 4
    n = rows * P
    shape = shape_with(axis, n, (3, 7))
    plan = cb.Plan(bd, n, partitions=P)
    info = plan.info()
    assert info["fullblock_seg" if axis == 0 else "fullblock_seg_strided"] >= 0
    b = synth.random_uniform(shape, seed=rows + axis)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    assert relerr(x, oracle.solve_axis(b.numpy(), axis, bd)) <= 1e-12
    f, _ = synth.random_modes(shape, seed=rows)
    lo, c = deriv_stencil(sch, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    assert relerr(out, oracle.apply_axis(f.numpy(), axis, bd, lo, c)) <= 1e-12


def test_partitioned_scratch_kept_by_the_plan(gpu):
    """cb_solve with P > 1 keeps its partition scratch in the plan, one buffer
    per stream: a larger call after a smaller one grows it, and calls
    alternating between two streams, which may overlap on the GPU, each use
    their own stream's buffer (all results exact)."""
    n, P = 1024, 8
    plan = cb.Plan(TRI, n, partitions=P)
    for other in ((2, 3), (40, 30), (2, 3)):
        b = synth.random_uniform(shape_with(0, n, other), seed=other[0])
        x = cb.solve(plan, b.to(gpu), 0).cpu().numpy()
        assert relerr(x, oracle.solve_axis(b.numpy(), 0, TRI)) <= 1e-12
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    bs = [synth.random_uniform(shape_with(1, n, (16, 8 + i)), seed=10 + i) for i in range(6)]
    bd = [b.to(gpu) for b in bs]
    outs = [torch.full_like(b, float("nan")) for b in bd]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    for i in range(6):
        cb.solve(plan, bd[i], 1, out=outs[i], stream=streams[i % 2])
    torch.cuda.synchronize()
    for b, o in zip(bs, outs):
        assert relerr(o.cpu().numpy(), oracle.solve_axis(b.numpy(), 1, TRI)) <= 1e-12
    # more streams than the plan keeps buffers for: it waits for the device
    # and releases them, then goes on allocating
    many = [torch.cuda.Stream() for _ in range(18)]
    b = synth.random_uniform(shape_with(2, n, (6, 5)), seed=99)
    ref = oracle.solve_axis(b.numpy(), 2, TRI)
    bd = b.to(gpu)
    outs = [torch.full_like(bd, float("nan")) for _ in many]
    for s, o in zip(many, outs):
        s.wait_stream(torch.cuda.current_stream())
        cb.solve(plan, bd, 2, out=o, stream=s)
    torch.cuda.synchronize()
    for o in outs:
        assert relerr(o.cpu().numpy(), ref) <= 1e-12
    plan.close()


def test_c3a_two_level_full_size(gpu):
    """64x64 lines of n = 8192 split into P = 16 workgroup partitions."""
    n = 8192
    shape = (64, 64, n)
    f, _ = synth.random_modes(shape, seed=3)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    b = oracle.stencil_axis(f.numpy(), 0, lo, c)
    plan = cb.Plan(TRI, n, partitions=16)
    x = cb.solve(plan, torch.from_numpy(b).to(gpu), 0).cpu().numpy()
    ref = oracle.solve_axis(b, 0, TRI)
    assert relerr(x, ref) <= 1e-12


# --------------------------------------------------------- precision modes --
@pytest.mark.parametrize("bands", ["tri", "penta"])
@pytest.mark.parametrize("axis", [0, 1])
def test_fp32_and_refinement(gpu, bands, axis):
    bd = TRI if bands == "tri" else PENTA
    n = 256
    shape = shape_with(axis, n, other=(16, 8))
    f, _ = synth.random_modes(shape, seed=7)
    lo, c = deriv_stencil(schemes.DERIV6 if bands == "tri" else schemes.DERIV10, n)
    ref = oracle.apply_axis(f.numpy(), axis, bd, lo, c)
    st = cb.Stencil(lo, c)
    p32 = cb.Plan(bd, n, precision="fp32")
    e32 = relerr(cb.apply_derivative(p32, st, f.to(gpu), axis).cpu().numpy(), ref)
    pr = cb.Plan(bd, n, precision="fp32_refine", refine_iters=2)
    er = relerr(cb.apply_derivative(pr, st, f.to(gpu), axis).cpu().numpy(), ref)
    print("fp32 %s: plain %.2e refined %.2e" % (bands, e32, er))
    assert er <= 1e-12
    assert e32 <= fp32_bound(bd)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bands", ["tri", "penta"])
@pytest.mark.parametrize("n,rpl", [(384, 12), (384, 0), (512, 16), (512, 8), (512, 0)])
def test_fp32_uniform_lanes(gpu, axis, bands, n, rpl):
    """Plain FP32 and FP32 + refinement (automatic count) on uniform lanes of
    8-16 rows, unit-stride and strided: the instances that read their
    kernel arguments at the point of use (12-16 rows, 8 with r = 2) and the
    ones that load them at entry, fused derivative against the oracle."""
    bd = TRI if bands == "tri" else PENTA
    f, _ = synth.random_modes(shape_with(axis, n, (6, 40)), seed=3 * n + axis)
    lo, c = deriv_stencil(schemes.DERIV6 if bands == "tri" else schemes.DERIV10, n)
    ref = oracle.apply_axis(f.numpy(), axis, bd, lo, c)
    st = cb.Stencil(lo, c)
    fd = f.to(gpu)
    for prec, tol in (("fp32_refine", 1e-12), ("fp32", fp32_bound(bd))):
        plan = cb.Plan(bd, n, precision=prec, rows_per_lane=rpl)
        info = plan.info()
        assert info["uniform"] == 1
        if rpl:
            assert info["rows_per_lane" if axis == 0 else "rows_per_lane_strided"] == rpl
        out = cb.apply_derivative(plan, st, fd, axis).cpu().numpy()
        plan.close()
        assert relerr(out, ref) <= tol, (prec, relerr(out, ref))


def fp32_bound(bands):
    """Error bound of a plain FP32 solve: 1e-6, the target, when the matrix
    allows it; else 2 kappa u, kappa the ratio of the extreme values of the
    band symbol a0 + 2 sum a_j cos(j t) (the cyclic matrix's condition number)
    and u = 2^-24.  Rounding the right-hand side to FP32 alone perturbs it by
    u, which the solve amplifies by up to kappa: the tenth-order pentadiagonal
    matrix has kappa = 2.1 / 0.1 = 21, so about 1.3e-6 is reachable there and
    no FP32 solve can promise 1e-6 (FP32 + refinement does, at 1e-12)."""
    r = (len(bands) - 1) // 2
    t = np.linspace(0.0, np.pi, 4097)
    f = bands[r] + sum(2 * bands[r + j] * np.cos(j * t) for j in range(1, r + 1))
    kappa = np.abs(f).max() / np.abs(f).min()
    return max(1e-6, 2 * kappa * 2.0 ** -24)


def test_refinement_ragged_solve(gpu):
    n = 613
    b = synth.random_uniform((4, 3, n), seed=1)
    plan = cb.Plan(PENTA, n, precision="fp32_refine", refine_iters=3)
    x = cb.solve(plan, b.to(gpu), 0).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), 0, PENTA)
    assert relerr(x, ref) <= 1e-12


# ------------------------------------------------------------- stencil -----
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rhs_stencil(gpu, axis):
    shape = (10, 14, 18)
    f = synth.random_uniform(shape, seed=axis)
    lo, c = schemes.stencil_deriv_collocated(schemes.DERIV10, 0.1)
    out = cb.rhs_stencil(cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.stencil_axis(f.numpy(), axis, lo, c)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()


# ----------------------------------------------------------- error paths ---
def test_errors_leave_output_untouched(gpu):
    plan = cb.Plan(TRI, 32)
    b = torch.ones((4, 4, 16), dtype=torch.float64, device=gpu)
    out = torch.full_like(b, 7.0)
    with pytest.raises(cb.CbError) as e:
        cb.solve(plan, b, 0, out=out)  # n mismatch
    assert e.value.status == cb.CB_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    host = cb.Plan(TRI, 16, host_only=True)
    with pytest.raises(cb.CbError):
        cb.solve(host, b, 0, out=out)


# --------------------------------------------- full sizes, every line ----
def full_check(f_dev, out_dev, axis, bands, lo, c):
    """Relative max error of a whole GPU output against the oracle's fused
    derivative of the whole grid (every line compared element by element)."""
    torch.cuda.synchronize()
    ref = oracle.apply_axis(f_dev.cpu().numpy(), axis, bands, lo, c)
    return relerr(out_dev.cpu().numpy(), ref)


def nan_like(t):
    """An output buffer prefilled with NaN, so an unwritten element fails."""
    return torch.full_like(t, float("nan"))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_headline_512_full_size(gpu, axis):
    """The benchmark's launch configuration on the full 512^3 grid, every line."""
    n = 512
    f, _ = synth.random_modes((n, n, n), seed=0, device=gpu)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    out = cb.apply_derivative(cb.Plan(TRI, n), cb.Stencil(lo, c), f, axis, out=nan_like(f))
    assert full_check(f, out, axis, TRI, lo, c) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c2_256_full_size(gpu, axis):
    """256^3: sixth-order derivative and collocated -> staggered interpolation."""
    n = 256
    f, _ = synth.random_modes((n, n, n), seed=2, device=gpu)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    out = cb.apply_derivative(cb.Plan(TRI, n), cb.Stencil(lo, c), f, axis, out=nan_like(f))
    assert full_check(f, out, axis, TRI, lo, c) <= 1e-12
    lo, c = schemes.stencil_interp_c2s(schemes.INTERP6)
    out = cb.apply_derivative(cb.Plan(INTERP, n), cb.Stencil(lo, c), f, axis, out=nan_like(f))
    assert full_check(f, out, axis, INTERP, lo, c) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_c3b_512_penta_full_size(gpu, axis):
    """512^3 tenth-order pentadiagonal derivative (z is the configuration's
    axis; x and y are what the benchmark times beside it)."""
    n = 512
    f, _ = synth.random_modes((n, n, n), seed=1, device=gpu)
    lo, c = deriv_stencil(schemes.DERIV10, n)
    out = cb.apply_derivative(cb.Plan(PENTA, n), cb.Stencil(lo, c), f, axis, out=nan_like(f))
    assert full_check(f, out, axis, PENTA, lo, c) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_headline_512_plain_solve_full_size(gpu, axis):
    """cb_solve on a 512^3 right-hand side (the benchmark's plain-solve lines)."""
    n = 512
    b = synth.random_uniform((n, n, n), seed=axis, device=gpu)
    x = cb.solve(cb.Plan(TRI, n), b, axis, out=nan_like(b))
    torch.cuda.synchronize()
    ref = oracle.solve_axis(b.cpu().numpy(), axis, TRI)
    assert relerr(x.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("P", [4, 7])
@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("xs", [1, 2])
def test_partitioned_fused_derivative(gpu, P, axis, xs):
    """Partitioned lines with the fused stencil; unit-stride rows direct (1) or staged (2)."""
    n = 96 * P
    shape = shape_with(axis, n, other=(5, 6))
    f, _ = synth.random_modes(shape, seed=P + axis)
    lo, c = deriv_stencil(schemes.DERIV10, n)
    plan = cb.Plan(PENTA, n, partitions=P, x_staging=xs)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), axis, PENTA, lo, c)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("n", [64, 500, 512, 613])
@pytest.mark.parametrize("xs", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_unit_stride_staging_paths(gpu, n, xs, prec):
    """Direct per-lane loads and the LDS-staged coalesced path give the same answer."""
    f, _ = synth.random_modes((6, 5, n), seed=n + xs)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    plan = cb.Plan(TRI, n, x_staging=xs, precision=prec)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), 0).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), 0, TRI, lo, c)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bands,n,rpl", [(TRI, 512, 16), (TRI, 613, 16), (PENTA, 384, 12), (PENTA, 512, 8)])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("interior", [1, 2])
def test_interior_solves(gpu, axis, bands, n, rpl, prec, interior):
    """Lane interiors by generalized PCR (1) or banded elimination (2) on every axis."""
    b = synth.random_uniform(shape_with(axis, n, (10, 18)), seed=n + axis + rpl)
    plan = cb.Plan(bands, n, rows_per_lane=rpl, interior=interior, precision=prec,
                   refine_iters=(3 if bands is PENTA else 2) if prec == "fp32_refine" else 0)
    assert plan.info()["interior_elimination"] == interior - 1
    out = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, bands)
    assert relerr(out, ref) <= 1e-12


def test_empty_grids(gpu):
    """Grids with no lines: every entry point succeeds and writes nothing."""
    lo, c = deriv_stencil(schemes.DERIV6, 64)
    st = cb.Stencil(lo, c)
    for P in (1, 2):
        plan = cb.Plan(TRI, 64, partitions=P)
        for shape, axis in (((3, 0, 64), 0), ((0, 64, 5), 1), ((64, 4, 0), 2)):
            f = torch.zeros(shape, dtype=torch.float64, device=gpu)
            out = torch.empty_like(f)
            cb.solve(plan, f, axis, out=out)
            cb.apply_derivative(plan, st, f, axis, out=out)
            cb.rhs_stencil(st, f, axis, out=out)
    torch.cuda.synchronize()


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bands,n", [(TRI, 512), (PENTA, 512), (TRI, 64), (TRI, 32), (PENTA, 1024)])
@pytest.mark.parametrize("fused", [False, True])
def test_thirty_two_rows_per_lane(gpu, axis, bands, n, fused):
    """32 rows per lane (uniform lanes, eliminated interiors) on every axis, including one- and two-lane lines."""
    plan = cb.Plan(bands, n, rows_per_lane=32)
    assert plan.info()["rows_per_lane"] == 32
    shape = shape_with(axis, n, (6, 40))
    if fused:
        f, _ = synth.random_modes(shape, seed=n + axis)
        lo, c = deriv_stencil(schemes.DERIV6 if bands is TRI else schemes.DERIV10, n)
        out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
        ref = oracle.apply_axis(f.numpy(), axis, bands, lo, c)
    else:
        b = synth.random_uniform(shape, seed=n + axis)
        out = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
        ref = oracle.solve_axis(b.numpy(), axis, bands)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bands,n", [(TRI, 512), (TRI, 613), (PENTA, 256), (PENTA, 500)])
def test_single_refinement_meets_tolerance(gpu, axis, bands, n):
    """One FP64 residual refinement of the FP32 reduction already meets 1e-12
    for these schemes (measured ~5e-14 tridiagonal, ~2.5e-13 pentadiagonal)."""
    f, _ = synth.random_modes(shape_with(axis, n, (8, 12)), seed=n + 7 * axis)
    lo, c = deriv_stencil(schemes.DERIV6 if bands is TRI else schemes.DERIV10, n)
    plan = cb.Plan(bands, n, precision="fp32_refine", refine_iters=1)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), axis, bands, lo, c)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 2])
def test_longest_one_partition_lines(gpu, axis):
    """n = 16384 in one workgroup per line (1024 lanes of 16 rows along x, 512
    lanes of 32 rows strided), on a few lines the oracle solves directly."""
    n = 16384
    plan = cb.Plan(TRI, n)
    i = plan.info()
    assert (i["lanes"], i["rows_per_lane"]) == (1024, 16)
    shape = shape_with(axis, n, (3, 2))
    b = synth.random_uniform(shape, seed=axis)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    ref = oracle.solve_axis(b.numpy(), axis, TRI)
    assert relerr(x, ref) <= 1e-12


@pytest.mark.parametrize("axis", [1, 2])
@pytest.mark.parametrize("bands", ["tri", "penta"])
def test_long_strided_lines_use_partitions(gpu, axis, bands):
    """n = 8192 strided lines run as 16 workgroup partitions (solve and fused derivative)."""
    bd = TRI if bands == "tri" else PENTA
    n = 8192
    plan = cb.Plan(bd, n)
    assert plan.info()["partitions_strided"] == 16
    shape = shape_with(axis, n, (5, 3))
    b = synth.random_uniform(shape, seed=axis)
    x = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
    assert relerr(x, oracle.solve_axis(b.numpy(), axis, bd)) <= 1e-12
    f, _ = synth.random_modes(shape, seed=axis + 1)
    lo, c = deriv_stencil(schemes.DERIV6 if bands == "tri" else schemes.DERIV10, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    assert relerr(out, oracle.apply_axis(f.numpy(), axis, bd, lo, c)) <= 1e-12


@pytest.mark.parametrize("axis", [1, 2])
@pytest.mark.parametrize("n", [96, 512, 613])
@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_tile_orders(gpu, axis, n, prec):
    """Strided tiles taken in launch order (1) or XCD-grouped order (2): the
    same lines are solved, bit for bit, with a tile count that is not a
    multiple of the XCD count and a partial last tile (407 lines)."""
    f, _ = synth.random_modes(shape_with(axis, n, (37, 11)), seed=n + axis)
    lo, c = deriv_stencil(schemes.DERIV6, n)
    fd = f.to(gpu)
    outs = []
    for order in (1, 2):
        plan = cb.Plan(TRI, n, precision=prec, tile_order=order)
        outs.append(cb.apply_derivative(plan, cb.Stencil(lo, c), fd, axis).cpu().numpy())
    ref = oracle.apply_axis(f.numpy(), axis, TRI, lo, c)
    assert relerr(outs[1], ref) <= 1e-12
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("scheme", ["deriv6", "deriv10", "interp6"])
@pytest.mark.parametrize("n", [64, 613, 2048, 8192])
def test_automatic_refinement_count_meets_tolerance(gpu, axis, scheme, n):
    """FP32 + refinement with the library's own iteration count (one for the
    sixth-order schemes, two for the tenth-order one) meets 1e-12, up to
    lines of 8192 rows."""
    bands = {"deriv6": TRI, "deriv10": PENTA, "interp6": INTERP}[scheme]
    plan = cb.Plan(bands, n, precision="fp32_refine")
    assert plan.info()["refine_iters"] == (2 if scheme == "deriv10" else 1)
    other = (4, 6) if n >= 2048 else (8, 12)
    shape = shape_with(axis, n, other)
    if scheme == "interp6":
        b = synth.random_uniform(shape, seed=n + axis)
        out = cb.solve(plan, b.to(gpu), axis).cpu().numpy()
        ref = oracle.solve_axis(b.numpy(), axis, bands)
    else:
        f, _ = synth.random_modes(shape, seed=n + 3 * axis)
        lo, c = deriv_stencil(schemes.DERIV6 if scheme == "deriv6" else schemes.DERIV10, n)
        out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
        ref = oracle.apply_axis(f.numpy(), axis, bands, lo, c)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("axis", [0, 2])
@pytest.mark.parametrize("bands,n", [(TRI, 32768), (PENTA, 20000)])
def test_lines_longer_than_a_workgroup(gpu, axis, bands, n):
    """Default plans for lines longer than 16384 rows split them into
    workgroup partitions by themselves (fused derivative, a few lines)."""
    plan = cb.Plan(bands, n)
    assert plan.info()["partitions"] == (n + 1023) // 1024
    f, _ = synth.random_modes(shape_with(axis, n, (3, 2)), seed=n + axis)
    lo, c = deriv_stencil(schemes.DERIV6 if bands is TRI else schemes.DERIV10, n)
    out = cb.apply_derivative(plan, cb.Stencil(lo, c), f.to(gpu), axis).cpu().numpy()
    ref = oracle.apply_axis(f.numpy(), axis, bands, lo, c)
    assert relerr(out, ref) <= 1e-12
