"""CPU checks of the host pre-factorisation (host-only plans, no GPU)."""
import numpy as np
import pytest

import oracle
from oracle import schemes
from paper_2101_02286_amd import cb, synth
from tests import plan_emulator

pytestmark = pytest.mark.filterwarnings("ignore")


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        cb.lib()
    except RuntimeError as e:
        pytest.skip(str(e))


def _bands(name):
    return dict(tri=[1 / 3, 1.0, 1 / 3], penta=schemes.bands_collocated(schemes.DERIV10),
                tri4=[0.25, 1.0, 0.25], interp=[0.3, 1.0, 0.3])[name]


def test_abi_exports_every_declared_symbol():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "cb.h")).read()
    declared = set(re.findall(r"\b(cb_[a-z_]+)\s*\(", hdr))
    declared -= {"cb_plan_t"}
    L = cb.lib()
    missing = [s for s in declared if not hasattr(L, s)]
    assert not missing, missing
    assert declared >= set(cb.ABI_SYMBOLS)


@pytest.mark.parametrize("name", ["tri", "penta"])
@pytest.mark.parametrize("n", [8, 11, 32, 37, 96, 192, 256, 512, 613, 1024])
@pytest.mark.parametrize("cyclic", [True, False])
def test_one_partition_plan_reproduces_oracle(name, n, cyclic):
    bands = _bands(name)
    p = cb.Plan(bands, n, cyclic=cyclic, host_only=True)
    b = np.random.default_rng(n).standard_normal((3, n))
    x = plan_emulator.solve(p, b)
    ref = oracle.solve_lines(b, bands, cyclic=cyclic)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("rpl", [4, 6, 8, 12, 16])
def test_rows_per_lane_choices(rpl):
    n = rpl * 32
    p = cb.Plan(_bands("penta"), n, rows_per_lane=rpl, host_only=True)
    assert p.info()["rows_per_lane"] == rpl
    b = np.random.default_rng(rpl).standard_normal((2, n))
    ref = oracle.solve_lines(b, _bands("penta"))
    assert np.abs(plan_emulator.solve(p, b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_per_row_bands():
    n, r = 300, 2
    bands = synth.random_bands(n, r, seed=4)
    p = cb.Plan(bands, n, per_row=True, host_only=True)
    assert not p.info()["uniform"]
    b = np.random.default_rng(0).standard_normal((2, n))
    ref = oracle.solve_lines(b, bands, per_row=True)
    assert np.abs(plan_emulator.solve(p, b) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("P", [2, 3, 4, 5, 7, 11, 15, 16])
@pytest.mark.parametrize("name", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [True, False])
def test_partitioned_plan_reproduces_oracle(P, name, cyclic):
    n = 64 * P + 13
    bands = _bands(name)
    p = cb.Plan(bands, n, partitions=P, cyclic=cyclic, host_only=True)
    b = np.random.default_rng(P).standard_normal((2, n))
    ref = oracle.solve_lines(b, bands, cyclic=cyclic)
    x = plan_emulator.solve(p, b)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("P,n", [(3, 3 * 40), (4, 4 * 512 + 5), (16, 8192)])
@pytest.mark.parametrize("name", ["tri", "penta"])
@pytest.mark.parametrize("cyclic", [True, False])
def test_boundary_rows_of_interior_inverse(P, n, name, cyclic):
    """Phase A's functionals: the first and last r rows of y_i = D_i^{-1} b_i
    from the plan's windowed boundary rows equal those of a dense solve of
    each interior block D_i (numpy), for random b."""
    bands = np.asarray(_bands(name))
    r = (len(bands) - 1) // 2
    p = cb.Plan(bands, n, partitions=P, cyclic=cyclic, host_only=True)
    K = p.info()["boundary_window"]
    ws = p.array(7).astype(int)
    assert 0 < K <= min(np.diff(ws)) - r
    b = np.random.default_rng(n + P).standard_normal((3, n))
    yf, yl = plan_emulator.boundary_values(p, b)
    for i in range(P):
        d0, d1 = ws[i] + r, ws[i + 1]
        N = d1 - d0
        D = np.zeros((N, N))
        for j in range(N):
            for o in range(-r, r + 1):
                if 0 <= j + o < N:
                    D[j, j + o] = bands[o + r]
        y = np.linalg.solve(D, b[:, d0:d1].T).T
        scale = np.abs(y).max()
        assert np.abs(yf[i] - y[:, :r]).max() <= 1e-14 * scale
        assert np.abs(yl[i] - y[:, N - r:]).max() <= 1e-14 * scale


@pytest.mark.parametrize("name", ["tri", "penta", "hept"])
@pytest.mark.parametrize("P,n", [(16, 8192), (8, 8192), (4, 1024)])
@pytest.mark.parametrize("seg_key", ["fullblock_seg", "fullblock_seg_strided"])
def test_full_block_segment(name, P, n, seg_key):
    """Phase C's full-block lane plan: a whole partition whose first r rows
    are identity equations (the interface values x~_i) and whose couplings to
    the next partition are moved to the right-hand side.  Solved by the
    emulated lane scheme with the middle lanes' coefficient block for every
    lane, lane 0's interface couplings and the last lane's forward coupling
    masked, it matches a dense solve of that block system."""
    bands = np.asarray(HEPT if name == "hept" else _bands(name))
    r = (len(bands) - 1) // 2
    p = cb.Plan(bands, n, partitions=P, host_only=True)
    seg = p.info()[seg_key]
    assert seg >= 0
    s = n // P
    rng = np.random.default_rng(s + r)
    b = rng.standard_normal((2, s))
    xi, xi1 = rng.standard_normal((2, r)), rng.standard_normal((2, r))
    v = b.copy()
    v[:, :r] = xi
    for c in range(r):  # row s-r+c couples to row s+c+o-r of the next partition
        for o in range(1, r + 1):
            if c + o >= r:
                v[:, s - r + c] -= bands[o + r] * xi1[:, c + o - r]
    D = np.zeros((s, s))
    for j in range(s):
        if j < r:
            D[j, j] = 1.0
            continue
        for o in range(-r, r + 1):
            if 0 <= j + o < s:
                D[j, j + o] = bands[o + r]
    ref = np.linalg.solve(D, v.T).T
    got = plan_emulator.solve_segment(p, v, seg)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # the masked form: every lane takes the middle block
    types = p.array(3, seg).astype(int)
    assert len(set(types[1:-1])) == 1


def test_boundary_window_is_short_for_compact_schemes():
    """The kept windows of the compact schemes' boundary rows (entries omitted
    below 2^-56 of the row's absolute sum): about 41 rows for alpha = 1/3, 68
    for the tenth-order pentadiagonal scheme, independent of the block size."""
    for name, lo, hi in (("tri", 35, 48), ("penta", 60, 76)):
        for n in (16 * 512, 16 * 2048):
            K = cb.Plan(_bands(name), n, partitions=16, host_only=True).info()["boundary_window"]
            assert lo <= K <= hi, (name, n, K)


HEPT = schemes.bands_collocated(schemes.DERIV12H)


@pytest.mark.parametrize("n", [7, 13, 24, 37, 96, 256, 300, 613, 1024])
@pytest.mark.parametrize("cyclic", [True, False])
@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_heptadiagonal_plans_reproduce_oracle(n, cyclic, P, precision):
    """r = 3 (Sec. 2's general band, Eq. (4)): the twelfth-order scheme's
    heptadiagonal matrix, every lane layout the plan picks (unit-stride and
    strided), one or several workgroup partitions."""
    if P > 1 and (precision != "fp64" or n < 9 * P):
        pytest.skip("partitioned plans are FP64 and need partitions of at least 3r rows")
    p = cb.Plan(HEPT, n, cyclic=cyclic, partitions=P, precision=precision, host_only=True)
    assert p.info()["r"] == 3
    b = np.random.default_rng(n + P).standard_normal((3, n))
    ref = oracle.solve_lines(b, HEPT, cyclic=cyclic)
    segs = [0]
    if P == 1 and p.info()["rows_per_lane_strided"] != p.info()["rows_per_lane"] or \
            p.info()["interior_elimination_strided"] != p.info()["interior_elimination"]:
        segs.append(1)
    for seg in segs:
        x = plan_emulator.solve(p, b, seg)
        assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max(), seg


def test_heptadiagonal_per_row_bands():
    n, r = 200, 3
    bands = synth.random_bands(n, r, seed=9)
    for cyclic in (True, False):
        p = cb.Plan(bands, n, per_row=True, cyclic=cyclic, host_only=True)
        b = np.random.default_rng(1).standard_normal((2, n))
        ref = oracle.solve_lines(b, bands, per_row=True, cyclic=cyclic)
        assert np.abs(plan_emulator.solve(p, b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_heptadiagonal_rejects_unbuilt_lane_sizes():
    with pytest.raises(cb.CbError):
        cb.Plan(HEPT, 96, rows_per_lane=12, host_only=True)
    with pytest.raises(cb.CbError):
        cb.Plan([0.0] * 4 + [1.0] + [0.0] * 4, 96, host_only=True)  # r = 4


def test_step_counts_match_paper():
    """Sec. 4: floor(log2 p) block-PCR steps; popcount(p)-1 detach steps."""
    for P in range(2, 34):
        info = cb.Plan([1 / 3, 1, 1 / 3], 40 * P, partitions=P, host_only=True).info()
        assert info["red_pcr_steps"] == P.bit_length() - 1, P
        assert info["red_detach_steps"] == bin(P).count("1") - 1, P
        sched = cb.Plan([1 / 3, 1, 1 / 3], 40 * P, partitions=P, host_only=True).schedule()
        # rows involved in detach/reattach: p - 2^floor(log2 p)
        assert sum(len(l) for l in sched) == P - (1 << (P.bit_length() - 1)), P


def test_eleven_row_example_schedule():
    """Sec. 3 worked example (Figs. 6-7): 11 rows -> row 11 detached, then 9, 10."""
    import os
    gold = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "reduced_schedule_paper.txt")):
        if line.startswith("example11"):
            _, k, v = line.split()
            gold[k] = v
    p = cb.Plan([1 / 3, 1, 1 / 3], 11 * 40, partitions=11, host_only=True)
    sched = [[d + 1 for d in lvl] for lvl in p.schedule()]  # 1-based as in the paper
    assert sched[0] == [int(v) for v in gold["detached_level0"].split(",")]
    assert sched[1] == [int(v) for v in gold["detached_level1"].split(",")]
    assert all(len(l) == 0 for l in sched[2:])
    info = p.info()
    assert info["red_pcr_steps"] == int(gold["pcr_steps"])
    assert info["red_detach_steps"] == int(gold["detach_steps"])


def test_interior_levels():
    """Sec. 4: ceil(log2 N_i) generalized-PCR steps for an interior block of N_i rows."""
    for n, rpl in ((512, 8), (512, 16), (384, 12), (96, 6)):
        info = cb.Plan([1 / 3, 1, 1 / 3], n, rows_per_lane=rpl, host_only=True).info()
        assert info["interior_levels"] == int(np.ceil(np.log2(rpl - 1)))
        assert info["lane_levels"] == int(np.log2(n // rpl))


def test_singular_matrix_rejected():
    with pytest.raises(cb.CbError) as e:
        cb.Plan([0.5, 1.0, 0.5], 64, host_only=True)
    assert e.value.status == cb.CB_ERR_SINGULAR
    cb.Plan([0.5, 1.0, 0.5], 63, host_only=True)  # odd n is regular


def test_bad_descriptors():
    with pytest.raises(cb.CbError) as e:
        cb.Plan([1.0, 2.0, 3.0, 4.0, 9.0, 6.0, 7.0, 8.0, 9.0], 64, host_only=True)  # r = 4
    assert e.value.status == cb.CB_ERR_UNSUPPORTED
    with pytest.raises(cb.CbError):
        cb.Plan([1 / 3, 1, 1 / 3], 2, host_only=True)
    with pytest.raises(cb.CbError):
        cb.Plan([1 / 3, 1, 1 / 3], 64, rows_per_lane=5, host_only=True)
    for order in (-1, 3):
        with pytest.raises(cb.CbError) as e:
            cb.Plan([1 / 3, 1, 1 / 3], 64, tile_order=order, host_only=True)
        assert e.value.status == cb.CB_ERR_INVALID_ARG
    for order in (0, 1, 2):
        cb.Plan([1 / 3, 1, 1 / 3], 64, tile_order=order, host_only=True)


def test_tuner_candidates_are_valid_layouts():
    from paper_2101_02286_amd import tune
    c = tune.candidates([1 / 3, 1.0, 1 / 3], 512, "fp64")
    rpls = {x["rows_per_lane"] for x in c}
    assert rpls == {8, 16, 4}  # 512 = 64 x 8 = 32 x 16 = 128 x 4 (6 and 12 do not divide into 2^k lanes)
    for x in c:
        L = 512 // x["rows_per_lane"]
        assert x["lines_per_wg"] * L <= 1024
    c5 = tune.candidates([1 / 20, 1 / 2, 1.0, 1 / 2, 1 / 20], 613, "fp32_refine")
    assert {x["rows_per_lane"] for x in c5} == {8, 16}  # ragged lines use the general layouts
    # strided rows: both tile orders, no unit-stride staging choice
    cs = tune.candidates([1 / 3, 1.0, 1 / 3], 512, "fp64", strided=True)
    assert {x["tile_order"] for x in cs} == {1, 2} and {x["x_staging"] for x in cs} == {0}
    cx = tune.candidates([1 / 3, 1.0, 1 / 3], 512, "fp64", strided=False)
    assert {x["tile_order"] for x in cx} == {0} and {x["x_staging"] for x in cx} == {1, 2}
    for x in cs[:8] + cx[:8]:
        cb.Plan([1 / 3, 1.0, 1 / 3], 512, host_only=True, **x).close()


def test_deep_levels_with_decayed_couplings():
    """Penta interior blocks of 510 rows: at deep generalized-PCR levels the
    couplings 2s apart decay to ~1e-37 and below; the factorisation must stay
    exact (equilibrated Eq. (6) systems, vacuous outer equations)."""
    n, P = 8192, 16
    bands = _bands("penta")
    p = cb.Plan(bands, n, partitions=P, host_only=True)
    b = np.random.default_rng(2).standard_normal((1, n))
    ref = oracle.solve_lines(b, bands)
    assert np.abs(plan_emulator.solve(p, b) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["tri", "penta"])
@pytest.mark.parametrize("n", [64, 256, 512, 1024])
def test_strided_layout_reproduces_oracle(name, n):
    """One-partition plans carry a second lane layout for strided launches."""
    bands = _bands(name)
    p = cb.Plan(bands, n, host_only=True)
    info = p.info()
    b = np.random.default_rng(n).standard_normal((2, n))
    ref = oracle.solve_lines(b, bands)
    two = (info["lanes_strided"] != info["lanes"]
           or info["interior_elimination_strided"] != info["interior_elimination"])
    for seg in ((0, 1) if two else (0,)):
        assert np.abs(plan_emulator.solve(p, b, seg) - ref).max() <= 1e-12 * np.abs(ref).max()
    if n == 512:
        assert (info["rows_per_lane"], info["rows_per_lane_strided"]) == (8, 32)
        # automatic interior solve: PCR for unit stride, elimination for strided
        assert (info["interior_elimination"], info["interior_elimination_strided"]) == (0, 1)
    assert p.array(11, 1 if two else 0)[6] == info["interior_elimination_strided"]


@pytest.mark.parametrize("name,n,rows", [("tri", 256, 8), ("tri", 512, 16), ("tri", 1024, 16), ("tri", 2048, 8),
                                         ("tri", 384, 12), ("tri", 500, 8), ("penta", 128, 8), ("penta", 256, 16),
                                         ("penta", 2048, 16), ("penta", 500, 8)])
def test_fp32_strided_rows_per_lane(name, n, rows):
    """FP32 plans lay strided lines out on uniform 16-row lanes where those
    measured fastest (r >= 2 from n = 256, r = 1 at n = 512..1024), else as
    before: 12 rows at n = 384, 8 rows for the other tridiagonal lengths and
    for general layouts (ragged n); and the layout still solves the system."""
    bands = _bands(name)
    p = cb.Plan(bands, n, precision="fp32_refine", host_only=True)
    info = p.info()
    assert info["rows_per_lane_strided"] == rows
    seg = 1 if (info["lanes_strided"] != info["lanes"] or
                info["interior_elimination_strided"] != info["interior_elimination"]) else 0
    b = np.random.default_rng(n).standard_normal((2, n))
    ref = oracle.solve_lines(b, bands)
    assert np.abs(plan_emulator.solve(p, b, seg) - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["tri", "penta"])
@pytest.mark.parametrize("n,rpl", [(512, 8), (512, 16), (384, 12), (613, 16), (200, 8), (512, 32), (64, 32),
                                   (32, 32)])
def test_interior_elimination_reproduces_oracle(name, n, rpl):
    """Lane interiors solved by banded elimination instead of generalized PCR."""
    bands = _bands(name)
    p = cb.Plan(bands, n, rows_per_lane=rpl, interior=2, host_only=True)
    assert p.info()["interior_elimination"] == 1
    b = np.random.default_rng(n + rpl).standard_normal((2, n))
    ref = oracle.solve_lines(b, bands)
    assert np.abs(plan_emulator.solve(p, b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_interior_elimination_rejected_where_unsupported():
    with pytest.raises(cb.CbError):
        cb.Plan([1 / 3, 1, 1 / 3], 512, rows_per_lane=4, interior=2, host_only=True)
    with pytest.raises(cb.CbError):
        cb.Plan([1 / 3, 1, 1 / 3], 8192, partitions=16, rows_per_lane=4, interior=2, host_only=True)


@pytest.mark.parametrize("name", ["tri", "penta"])
@pytest.mark.parametrize("n,P,interior", [(8192, 16, 0), (8192, 16, 1), (8192, 16, 2), (1000, 3, 0), (4099, 7, 0)])
def test_partition_interiors(name, n, P, interior):
    """Workgroup partitions solve their lane interiors by elimination by
    default (PCR on request); either way the plan reproduces the oracle."""
    bands = _bands(name)
    p = cb.Plan(bands, n, partitions=P, interior=interior, host_only=True)
    assert p.info()["interior_elimination"] == (0 if interior == 1 else 1)
    b = np.random.default_rng(n + P).standard_normal((2, n))
    ref = oracle.solve_lines(b, bands)
    assert np.abs(plan_emulator.solve(p, b) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_tuner_searches_partition_counts_for_long_lines():
    from paper_2101_02286_amd import tune
    c = tune.candidates([1 / 3, 1.0, 1 / 3], 8192, "fp64")
    parts = {x["partitions"] for x in c}
    assert {2, 4, 8, 16} <= parts
    for x in c:  # every candidate builds
        cb.Plan([1 / 3, 1.0, 1 / 3], 8192, host_only=True, **x).close()
    assert {x["partitions"] for x in tune.candidates([1 / 3, 1.0, 1 / 3], 512, "fp64")} == {1}
    assert {x["partitions"] for x in tune.candidates([1 / 3, 1.0, 1 / 3], 8192, "fp32_refine")} == {1}


def test_thirty_two_rows_need_uniform_elimination():
    with pytest.raises(cb.CbError):  # ragged: general layout
        cb.Plan([1 / 3, 1.0, 1 / 3], 500, rows_per_lane=32, host_only=True)
    with pytest.raises(cb.CbError):  # generalized PCR interiors are not built for 32 rows
        cb.Plan([1 / 3, 1.0, 1 / 3], 512, rows_per_lane=32, interior=1, host_only=True)
    i = cb.Plan([1 / 3, 1.0, 1 / 3], 512, rows_per_lane=32, host_only=True).info()
    assert (i["lanes"], i["rows_per_lane"], i["interior_elimination"]) == (16, 32, 1)


def test_long_lines_split_strided_launches():
    """One-partition plans with n > 4096, and ragged ones (general layouts) of
    1025..4096 rows in FP64 or 2049..4096 in FP32, solve strided lines in
    ~512-row workgroup partitions (unit-stride lines stay whole)."""
    tri = [1 / 3, 1.0, 1 / 3]
    assert cb.Plan(tri, 4096, host_only=True).info()["partitions_strided"] == 1
    assert cb.Plan(tri, 2048, host_only=True).info()["partitions_strided"] == 1
    assert cb.Plan(tri, 1024, host_only=True).info()["partitions_strided"] == 1
    assert cb.Plan(tri, 1000, host_only=True).info()["partitions_strided"] == 1
    for n, P in ((1025, 3), (1100, 3), (2000, 4), (4000, 8)):
        i = cb.Plan(tri, n, host_only=True).info()
        assert (i["partitions"], i["partitions_strided"]) == (1, P)
    assert cb.Plan(tri, 2048, cyclic=False, host_only=True).info()["partitions_strided"] == 4
    # FP32: from 4097 rows, and from 2049 on general layouts
    for n, P in ((1100, 1), (2048, 1), (2500, 5), (4096, 1), (5000, 10)):
        assert cb.Plan(tri, n, precision="fp32_refine", host_only=True).info()["partitions_strided"] == P
    i = cb.Plan(tri, 8192, host_only=True).info()
    assert (i["partitions"], i["partitions_strided"]) == (1, 16)
    # lines longer than one workgroup holds are partitioned plans already
    i = cb.Plan(tri, 32768, host_only=True).info()
    assert (i["partitions"], i["partitions_strided"]) == (32, 32)
    assert cb.Plan(tri, 8192, precision="fp32_refine", host_only=True).info()["partitions_strided"] == 16
    assert cb.Plan(tri, 8192, rows_per_lane=16, host_only=True).info()["partitions_strided"] == 1


def test_automatic_refinement_count():
    """CB_FP32_REFINE with refine_iters 0: the fewest k >= 1 with
    (kappa u)^(k+1) <= 1e-13, u = 2^-24, kappa the ratio of the extreme values
    of the symbol a0 + 2 sum a_j cos(j t) (cyclic: the eigenvalues)."""
    u = 2.0 ** -24

    def expect(bands, n, cyclic):
        r = (len(bands) - 1) // 2
        t = 2 * np.pi * np.arange(n) / n if cyclic else np.linspace(0, np.pi, 65537)
        f = bands[r] + sum(2 * bands[r + j] * np.cos(j * t) for j in range(1, r + 1))
        ku = np.abs(f).max() / np.abs(f).min() * u
        k = 1
        while ku ** (k + 1) > 1e-13 and k < 8:
            k += 1
        return k

    tri = [1 / 3, 1.0, 1 / 3]                      # kappa 5: (5u)^2 = 8.9e-14
    penta = [1 / 20, 1 / 2, 1.0, 1 / 2, 1 / 20]    # kappa 21: (21u)^2 = 1.6e-12
    interp = [0.3, 1.0, 0.3]                       # kappa 4
    weak = [0.49, 1.0, 0.49]                       # kappa 99: (99u)^2 = 3.5e-11
    for bands, n, cyc, want in ((tri, 512, 1, 1), (tri, 613, 0, 1), (penta, 512, 1, 2), (penta, 100, 0, 2),
                                (interp, 256, 1, 1), (weak, 512, 1, 2)):
        assert expect(bands, n, cyc) == want
        p = cb.Plan(bands, n, cyclic=bool(cyc), precision="fp32_refine", host_only=True)
        assert p.info()["refine_iters"] == want, (bands, n, cyc)
    # explicit counts are kept; per-row and unsymmetric bands take 2
    assert cb.Plan(tri, 512, precision="fp32_refine", refine_iters=3, host_only=True).info()["refine_iters"] == 3
    rows = np.tile(np.array(tri), (64, 1))
    assert cb.Plan(rows, 64, per_row=True, precision="fp32_refine", host_only=True).info()["refine_iters"] == 2
    assert cb.Plan([0.2, 1.0, 0.3], 64, precision="fp32_refine", host_only=True).info()["refine_iters"] == 2
    assert cb.Plan(tri, 512, precision="fp64", host_only=True).info()["refine_iters"] == 0


def test_automatic_partition_count():
    """partitions 0: one workgroup per line up to 16384 rows in FP64 (8192 in
    FP32), else ceil(n / 1024) workgroup partitions (at most 64)."""
    tri = [1 / 3, 1.0, 1 / 3]
    for n, want in ((512, 1), (16384, 1), (16385, 17), (32768, 32), (50000, 49), (100000, 64)):
        info = cb.Plan(tri, n, host_only=True).info()
        assert info["partitions"] == want, n
    assert cb.Plan(tri, 32768, partitions=4, host_only=True).info()["partitions"] == 4
    for n, want in ((8192, 1), (8193, 9), (32768, 32)):
        info = cb.Plan(tri, n, precision="fp32_refine", host_only=True).info()
        assert info["partitions"] == want and info["refine_iters"] == 1, n


@pytest.mark.parametrize("n", [512, 8192])
def test_generalized_pcr_on_request_without_row_count(n):
    """interior = 1 without rows_per_lane: every layout of the plan uses
    generalized PCR (strided lanes stop at 16 rows, since 32-row lanes only
    eliminate)."""
    p = cb.Plan([1 / 3, 1.0, 1 / 3], n, interior=1, host_only=True)
    info = p.info()
    assert info["interior_elimination"] == 0 and info["interior_elimination_strided"] == 0
    assert info["rows_per_lane_strided"] <= 16


def test_batch_tuner_candidates_are_valid_plans():
    """Every choice the batch tuner would time builds a host-only plan, and
    the strided and unit-stride sets differ only in the layout knob."""
    from paper_2101_02286_amd import tune
    tri = schemes.bands_collocated(schemes.DERIV6)
    penta = schemes.bands_collocated(schemes.DERIV10)
    for bands, n, prec in ((tri, 384, "fp32_refine"), (penta, 64, "fp64"), (tri, 1000, "fp64")):
        for strided in (False, True):
            cands = tune.batch_candidates(bands, n, prec, 0, strided)
            assert cands
            for c in cands:
                assert ("tile_order" in c) == strided and ("block_barriers" in c) != strided
                cb.Plan(bands, n, precision=prec, host_only=True, **c).close()
