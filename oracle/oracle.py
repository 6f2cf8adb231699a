"""ctypes wrapper around the FP64 C oracle (cb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Arrays are numpy float64 in C order.  A 3D field has shape (nz, ny, nx) with
x the unit-stride index; `axis` 0/1/2 means x/y/z.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cb_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liborc.so")
_lib = None


def build(force=False):
    """Compile the oracle with gcc (OpenMP over lines)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        I64P = ctypes.POINTER(ctypes.c_int64)
        lib.orc_solve_lines.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int64, P, P]
        lib.orc_stencil_axis.argtypes = [I64P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        lib.orc_solve_axis.argtypes = [I64P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_apply_axis.argtypes = [I64P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, P, P, P]
        lib.orc_matvec_axis.argtypes = [I64P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_num_threads.argtypes = []
        for f in ("orc_solve_lines", "orc_stencil_axis", "orc_solve_axis", "orc_apply_axis",
                  "orc_matvec_axis", "orc_num_threads"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(f):
    if f.ndim != 3:
        raise ValueError("expected a (nz, ny, nx) array")
    nz, ny, nx = f.shape
    return (ctypes.c_int64 * 3)(nx, ny, nz)


def _check(st):
    if st == 3:
        raise OracleError("singular system")
    if st != 0:
        raise OracleError("bad argument (status %d)" % st)


def _bands(bands, r, n, per_row):
    b = _f64(bands)
    w = 2 * r + 1
    if per_row:
        if b.size != n * w:
            raise ValueError("per-row bands need n*(2r+1) values")
    elif b.size != w:
        raise ValueError("constant bands need 2r+1 values")
    return b


def solve_lines(b, bands, cyclic=True, per_row=False):
    """x = A^{-1} b for every row of a (lines, n) array."""
    b = _f64(b)
    if b.ndim == 1:
        b = b[None, :]
    nl, n = b.shape
    bands = np.asarray(bands, dtype=np.float64)
    r = (bands.shape[-1] - 1) // 2
    bands = _bands(bands, r, n, per_row)
    x = np.empty_like(b)
    _check(_load().orc_solve_lines(r, n, _dp(bands), int(per_row), int(cyclic), nl, _dp(b), _dp(x)))
    return x


def solve_axis(b, axis, bands, cyclic=True, per_row=False):
    """x = A^{-1} b along `axis` of a (nz, ny, nx) array."""
    b = _f64(b)
    bands = np.asarray(bands, dtype=np.float64)
    r = (bands.shape[-1] - 1) // 2
    n = b.shape[2 - axis]
    bands = _bands(bands, r, n, per_row)
    x = np.empty_like(b)
    _check(_load().orc_solve_axis(_dims(b), axis, r, _dp(bands), int(per_row), int(cyclic), _dp(b), _dp(x)))
    return x


def stencil_axis(f, axis, lo, coefs):
    """out_j = sum_q coefs[q-lo] f_{(j+q) mod n} along `axis` (periodic)."""
    f = _f64(f)
    c = _f64(coefs)
    out = np.empty_like(f)
    _check(_load().orc_stencil_axis(_dims(f), axis, lo, lo + c.size - 1, _dp(c), _dp(f), _dp(out)))
    return out


def apply_axis(f, axis, bands, lo, coefs, cyclic=True):
    """Compact operator A^{-1} B f along `axis` (derivative or interpolation)."""
    f = _f64(f)
    c = _f64(coefs)
    bands = np.asarray(bands, dtype=np.float64)
    r = (bands.size - 1) // 2
    out = np.empty_like(f)
    _check(_load().orc_apply_axis(_dims(f), axis, r, _dp(bands), int(cyclic), lo, lo + c.size - 1,
                                  _dp(c), _dp(f), _dp(out)))
    return out


def matvec_axis(x, axis, bands, cyclic=True, per_row=False):
    """y = A x along `axis` (banded, periodic when cyclic)."""
    x = _f64(x)
    bands = np.asarray(bands, dtype=np.float64)
    r = (bands.shape[-1] - 1) // 2
    n = x.shape[2 - axis]
    bands = _bands(bands, r, n, per_row)
    y = np.empty_like(x)
    _check(_load().orc_matvec_axis(_dims(x), axis, r, _dp(bands), int(per_row), int(cyclic), _dp(x), _dp(y)))
    return y


def num_threads():
    return _load().orc_num_threads()
