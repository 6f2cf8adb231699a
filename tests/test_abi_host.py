"""C ABI argument checking that needs no GPU: every rejected call must return
an error status (and a message) before anything touches the device."""
import ctypes

import pytest

from paper_2101_02286_amd import cb


@pytest.fixture(scope="module")
def L():
    try:
        return cb.lib()
    except RuntimeError as e:
        pytest.skip(str(e))


def grid(n=(16, 8, 4)):
    g = cb.Grid()
    g.n[0], g.n[1], g.n[2] = n
    g.stride[0], g.stride[1], g.stride[2] = 1, n[0], n[0] * n[1]
    return g


def test_solve_rejects_host_only_plan(L):
    p = cb.Plan([1 / 3, 1, 1 / 3], 16, host_only=True)
    g = grid()
    st = L.cb_solve(p.h, ctypes.byref(g), 0, ctypes.c_void_p(64), ctypes.c_void_p(1 << 20), None)
    assert st == cb.CB_ERR_INVALID_ARG
    assert b"host-only" in L.cb_last_error()


def test_null_and_bad_arguments(L):
    g = grid()
    assert L.cb_solve(None, ctypes.byref(g), 0, None, None, None) == cb.CB_ERR_INVALID_ARG
    st = cb.Stencil(-1, [1.0, 2.0, 3.0])
    assert L.cb_rhs_stencil(ctypes.byref(st.c), ctypes.byref(g), 3, ctypes.c_void_p(64),
                            ctypes.c_void_p(1 << 20), None) == cb.CB_ERR_INVALID_ARG
    bad = cb.StencilC(-4, 0, (ctypes.c_double * 7)())
    assert L.cb_rhs_stencil(ctypes.byref(bad), ctypes.byref(g), 0, ctypes.c_void_p(64),
                            ctypes.c_void_p(1 << 20), None) == cb.CB_ERR_INVALID_ARG
    g0 = grid((0, 8, 4))  # empty along the solve axis
    assert L.cb_rhs_stencil(ctypes.byref(st.c), ctypes.byref(g0), 0, ctypes.c_void_p(64),
                            ctypes.c_void_p(1 << 20), None) == cb.CB_ERR_INVALID_ARG
    gneg = grid((16, 8, 4))
    gneg.n[1] = -1
    assert L.cb_rhs_stencil(ctypes.byref(st.c), ctypes.byref(gneg), 0, ctypes.c_void_p(64),
                            ctypes.c_void_p(1 << 20), None) == cb.CB_ERR_INVALID_ARG
    # overlapping input and output
    assert L.cb_rhs_stencil(ctypes.byref(st.c), ctypes.byref(g), 0, ctypes.c_void_p(4096),
                            ctypes.c_void_p(4096 + 8), None) == cb.CB_ERR_INVALID_ARG
    assert b"overlap" in L.cb_last_error()


def test_batch_rejects_bad_workspace(L):
    items = (cb.BatchItem * 1)()
    assert L.cb_batch_build(items, 1, None, 0, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_batch_build(items, 1, ctypes.c_void_p(4096), 16, None) == cb.CB_ERR_INVALID_ARG
    assert L.cb_batch_launch(ctypes.c_void_p(12345), 0, None) == cb.CB_ERR_INVALID_ARG


def test_plan_info_of_host_plan(L):
    p = cb.Plan([1 / 20, 1 / 2, 1, 1 / 2, 1 / 20], 8192, partitions=16, host_only=True)
    i = p.info()
    assert (i["r"], i["n"], i["partitions"], i["lanes"], i["rows_per_lane"]) == (2, 8192, 16, 64, 8)
    assert i["red_pcr_steps"] == 4 and i["red_detach_steps"] == 0
    assert i["device_bytes"] == 0


def test_empty_grid_is_a_noop(L):
    """A grid with no lines succeeds and launches nothing (so it needs no GPU)."""
    st = cb.Stencil(-1, [1.0, 2.0, 3.0])
    for n, axis in (((16, 0, 4), 0), ((0, 8, 4), 1), ((16, 8, 0), 0)):
        g = grid(n)
        g.stride[0], g.stride[1], g.stride[2] = 1, 16, 128
        assert L.cb_rhs_stencil(ctypes.byref(st.c), ctypes.byref(g), axis, ctypes.c_void_p(64),
                                ctypes.c_void_p(1 << 20), None) == cb.CB_OK
