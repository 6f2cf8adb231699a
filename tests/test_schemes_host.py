"""The callers' scheme table (paper_2101_02286_amd/schemes.py, used by the
benchmark and the server) equals the oracle's pinned one (oracle/schemes.py,
checked against closed forms, the paper's printed values and exact Taylor
conditions in test_oracle_pins.py), for several line lengths."""
import math

import numpy as np
import pytest

from oracle import schemes as osch
from paper_2101_02286_amd import schemes as psch


def _close(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return a.shape == b.shape and np.allclose(a, b, rtol=4e-16, atol=0.0)


@pytest.mark.parametrize("n", [32, 100, 256, 613, 8192])
def test_derivative_schemes_match_pinned(n):
    h = 2 * math.pi / n
    for name, s in (("tri6", osch.DERIV6), ("penta10", osch.DERIV10), ("hept12", osch.DERIV12H)):
        assert _close(psch.bands(name), osch.bands_collocated(s)), name
        lo_p, c_p = psch.stencil(name, n)
        lo_o, c_o = osch.stencil_deriv_collocated(s, h)
        assert lo_p == lo_o and _close(c_p, c_o), name


@pytest.mark.parametrize("n", [32, 256, 1000])
def test_staggered_schemes_match_pinned(n):
    h = 2 * math.pi / n
    for name, s in (("interp6", osch.INTERP6), ("stag6", osch.STAG6)):
        assert _close(psch.bands(name), [float(s["alpha"]), 1.0, float(s["alpha"])]), name
    assert psch.stencil("interp6", n, "c2s") == osch.stencil_interp_c2s(osch.INTERP6)
    assert psch.stencil("interp6", n, "s2c") == osch.stencil_interp_s2c(osch.INTERP6)
    for grid, ref in (("c2s", osch.stencil_deriv_c2s), ("s2c", osch.stencil_deriv_s2c)):
        lo_p, c_p = psch.stencil("stag6", n, grid)
        lo_o, c_o = ref(osch.STAG6, h)
        assert lo_p == lo_o and _close(c_p, c_o), grid


def test_server_and_benchmark_use_the_table():
    """The server's plans and stencils come from the same table."""
    import bench
    st = bench.scheme_stencil("penta10", 512)
    lo, c = osch.stencil_deriv_collocated(osch.DERIV10, 2 * math.pi / 512)
    assert st.lo == lo and _close(st.coefs, c)
