"""GPU tests of the autotuners: every launch choice they time and keep must
give the oracle's result, and the batch tuner must keep plans per group."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import schemes
from paper_2101_02286_amd import cb, synth, tune

pytestmark = pytest.mark.gpu

TRI = schemes.bands_collocated(schemes.DERIV6)
PENTA = schemes.bands_collocated(schemes.DERIV10)


def relerr(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def stencil(scheme, n):
    lo, c = schemes.stencil_deriv_collocated(scheme, 2 * math.pi / n)
    return cb.Stencil(lo, c), lo, c


@pytest.mark.parametrize("axis", [0, 2])
def test_tune_single_problem(gpu, axis):
    """tune.tune over the first candidates of one problem: the table holds
    what it timed, the best is among them, and the tuned plan is exact."""
    n = 128
    shape = (n, 8, 8) if axis == 2 else (8, 8, n)
    f, _ = synth.random_modes(shape, seed=5, device=gpu)
    st, lo, c = stencil(schemes.DERIV6, n)
    best, table = tune.tune(TRI, n, f, axis, stencil=st, reps=2, cache=None, max_candidates=12)
    assert table and all(r["ms"] > 0 for r in table)
    fastest = min(table, key=lambda r: r["ms"])
    assert all(best[k] == fastest[k] for k in best)
    plan = tune.tuned_plan(TRI, n, f, axis, stencil=st, reps=2, cache=None, max_candidates=12)
    out = cb.apply_derivative(plan, st, f, axis).cpu().numpy()
    ref = oracle.apply_axis(f.cpu().numpy(), axis, TRI, lo, c)
    assert relerr(out, ref) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_tune_batch_keeps_exact_plans(gpu, precision):
    """tune.tune_batch on a small uneven batch (tri- and pentadiagonal items,
    unit-stride and strided rows): the kept plans give the oracle's result
    for every item, and items of different line lengths get their own plans."""
    grids = [(48, 40, 24), (96, 32, 16)]
    items, refs = [], []
    for gi, (nx, ny, nz) in enumerate(grids):
        f, _ = synth.random_modes((nz, ny, nx), seed=20 + gi, device=gpu)
        for ax, bands, scheme in ((0, TRI, schemes.DERIV6), (1, PENTA, schemes.DERIV10), (2, TRI, schemes.DERIV6)):
            n = f.shape[2 - ax]
            st, lo, c = stencil(scheme, n)
            out = torch.full_like(f, float("nan"))
            items.append((bands, st, f, out, ax))
            refs.append(oracle.apply_axis(f.cpu().numpy(), ax, bands, lo, c))
    plans, choices, res = tune.tune_batch(items, precision=precision, reps=2, max_candidates=4)
    assert len(plans) == len(items) and len(choices) == 6
    assert res["candidates_timed"] > 0
    assert res["tuned_ms"] > 0 and res["automatic_ms"] > 0
    batch = cb.Batch([(p, st, f, o, ax) for p, (_b, st, f, o, ax) in zip(plans, items)])
    batch.launch()
    torch.cuda.synchronize()
    for (_b, _st, _f, o, _ax), ref in zip(items, refs):
        assert relerr(o.cpu().numpy(), ref) <= 1e-12
    # items 0 and 3 are both unit-stride tridiagonal lines but of different n
    assert plans[0] is not plans[3]
    for p in {id(p): p for p in plans}.values():
        p.close()
