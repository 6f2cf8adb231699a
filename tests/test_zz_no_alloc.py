"""cb_solve_noalloc (the allocation-free variant of cb_solve) against cb_solve.

Both run the same kernels, so their outputs must be bitwise equal; the
variant only takes its partition scratch from the library's fixed per-GPU
array.  Each case makes two calls in a row, the second with a smaller input
(the array keeps the first call's contents), on partitioned lines (P > 1)
along x, y and z and on the strided partitioned launch of a long
one-partition FP64 line.  The oracle checks the values too (FP64: 1e-12).
"""
import numpy as np
import pytest

import oracle
from oracle import schemes
from paper_2101_02286_amd import cb

pytestmark = pytest.mark.gpu

TRI = [1 / 3, 1.0, 1 / 3]
PENTA = schemes.bands_collocated(schemes.DERIV10)


def _pair(plan, b, axis):
    import torch
    x_ref = torch.full_like(b, float("nan"))
    x_na = torch.full_like(b, float("nan"))
    cb.solve(plan, b, axis, out=x_ref)
    cb.solve_noalloc(plan, b, axis, out=x_na)
    torch.cuda.synchronize()
    return x_ref, x_na


def _check(plan, bands, shape, axis, seed, dev):
    import torch
    rng = np.random.default_rng(seed)
    b = torch.from_numpy(rng.uniform(-1, 1, shape)).to(dev)
    x_ref, x_na = _pair(plan, b, axis)
    assert torch.equal(x_ref, x_na), "noalloc differs from cb_solve"
    # oracle on a few lines (the whole output for small grids)
    bn = b.cpu().numpy()
    lines = np.moveaxis(bn, 2 - axis, -1).reshape(-1, bn.shape[2 - axis])
    pick = np.linspace(0, lines.shape[0] - 1, min(lines.shape[0], 64)).astype(int)
    ref = oracle.solve_lines(lines[pick], bands, cyclic=plan.cyclic)
    got = np.moveaxis(x_na.cpu().numpy(), 2 - axis, -1).reshape(-1, bn.shape[2 - axis])[pick]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("name,bands", [("tri", TRI), ("penta", PENTA)])
def test_noalloc_partitioned_matches_cb_solve(gpu, axis, name, bands):
    n = 2048
    plan = cb.Plan(bands, n, partitions=8)
    shape_big = [24, 20, 16]
    shape_big[2 - axis] = n
    shape_small = [6, 5, 4]
    shape_small[2 - axis] = n
    print("noalloc case", name, "axis", axis, "shapes", shape_big, shape_small, flush=True)
    _check(plan, bands, tuple(shape_big), axis, 1, gpu)
    _check(plan, bands, tuple(shape_small), axis, 2, gpu)
    plan.close()


def test_noalloc_strided_long_line(gpu):
    """n > 4096 FP64 one-partition plan: strided launches split the lines into
    workgroup partitions and use the scratch; unit-stride ones do not."""
    n = 6000
    plan = cb.Plan(TRI, n)
    assert plan.info()["partitions_strided"] > 1
    print("noalloc strided long line n", n, flush=True)
    _check(plan, TRI, (n, 12, 10), 2, 3, gpu)
    _check(plan, TRI, (n, 3, 2), 2, 4, gpu)
    _check(plan, TRI, (3, 2, n), 0, 5, gpu)
    plan.close()


def test_noalloc_acyclic_and_non_power_of_two(gpu):
    n = 3000
    plan = cb.Plan(PENTA, n, partitions=5, cyclic=False)
    print("noalloc acyclic P=5", flush=True)
    _check(plan, PENTA, (7, 9, n), 0, 6, gpu)
    _check(plan, PENTA, (2, 3, n), 0, 7, gpu)
    plan.close()


def test_noalloc_rejects_scratch_beyond_limit(gpu):
    """A solve needing more scratch than the fixed array is refused before
    anything is enqueued; its output stays untouched."""
    import torch
    P = 16
    n = 8 * P
    plan = cb.Plan(TRI, n, partitions=P)
    per_line = P * 3 * 1 * 8
    nlines = cb.NOALLOC_SCRATCH_BYTES // per_line + 1
    ny = 64
    nz = (nlines + ny - 1) // ny
    print("noalloc limit lines", nz * ny, flush=True)
    b = torch.zeros((nz, ny, n), dtype=torch.float64, device=gpu)
    x = torch.full_like(b, 7.0)
    with pytest.raises(cb.CbError) as ei:
        cb.solve_noalloc(plan, b, 0, out=x)
    assert ei.value.status == cb.CB_ERR_UNSUPPORTED
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((x == 7.0).all())
    # a part of the same grid that fits still solves
    xs = cb.solve_noalloc(plan, b[:2], 0, out=x[:2])
    torch.cuda.synchronize()
    assert bool((xs == 0.0).all())
    plan.close()
