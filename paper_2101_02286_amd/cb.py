"""Thin ctypes binding of libcb.so (the C ABI declared in include/cb.h).

Only argument marshalling happens here: every step of a solve runs in the
library's HIP kernels.  Device arrays are torch tensors (float64, on a ROCm
device); PyTorch provides memory and streams only.  The library is loaded on
first use and a missing library is an error (there is no fallback).
"""
import ctypes
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcb.so")
_lib = None

CB_OK, CB_ERR_INVALID_ARG, CB_ERR_UNSUPPORTED, CB_ERR_SINGULAR, CB_ERR_OOM, CB_ERR_HIP = range(6)
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32_refine": 2}
ABI_SYMBOLS = ("cb_plan", "cb_plan_destroy", "cb_rhs_stencil", "cb_solve", "cb_apply_derivative",
               "cb_solve_noalloc", "cb_copy_lines",
               "cb_batch_workspace_size", "cb_batch_workspace_bytes", "cb_batch_build", "cb_batch_launch", "cb_solve_batched",
               "cb_plan_get_info",
               "cb_plan_get_schedule", "cb_plan_get_array", "cb_last_error")


class CbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libcb status %d: %s" % (status, msg))
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int32), ("n", ctypes.c_int32), ("bands", ctypes.POINTER(ctypes.c_double)),
                ("per_row", ctypes.c_int32), ("cyclic", ctypes.c_int32), ("partitions", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refine_iters", ctypes.c_int32),
                ("rows_per_lane", ctypes.c_int32), ("host_only", ctypes.c_int32),
                ("lines_per_wg", ctypes.c_int32), ("block_barriers", ctypes.c_int32),
                ("x_staging", ctypes.c_int32), ("interior", ctypes.c_int32),
                ("tile_order", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64 * 3), ("stride", ctypes.c_int64 * 3)]


class StencilC(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32), ("hi", ctypes.c_int32), ("coef", ctypes.c_double * 7)]


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("stencil", ctypes.POINTER(StencilC)), ("grid", Grid),
                ("axis", ctypes.c_int32), ("inp", ctypes.c_void_p), ("out", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in
                ("r", "n", "cyclic", "precision", "refine_iters", "partitions", "lanes", "rows_per_lane",
                 "uniform", "interior_levels", "lane_levels", "red_phases", "red_pcr_steps",
                 "red_detach_steps")] + [("device_bytes", ctypes.c_int64),
                                         ("rows_per_lane_strided", ctypes.c_int32),
                                         ("lanes_strided", ctypes.c_int32),
                                         ("interior_elimination", ctypes.c_int32),
                                         ("interior_elimination_strided", ctypes.c_int32),
                                         ("partitions_strided", ctypes.c_int32),
                                         ("boundary_window", ctypes.c_int32),
                                         ("fullblock_seg", ctypes.c_int32),
                                         ("fullblock_seg_strided", ctypes.c_int32)]


def lib():
    """Load libcb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libcb.so is not built (run python -m paper_2101_02286_amd.build): %s"
                               % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.cb_plan.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
        L.cb_plan_destroy.argtypes = [vp]
        L.cb_rhs_stencil.argtypes = [ctypes.POINTER(StencilC), ctypes.POINTER(Grid), i32, vp, vp, vp]
        L.cb_solve.argtypes = [vp, ctypes.POINTER(Grid), i32, vp, vp, vp]
        L.cb_solve_noalloc.argtypes = [vp, ctypes.POINTER(Grid), i32, vp, vp, vp]
        L.cb_copy_lines.argtypes = [vp, ctypes.POINTER(Grid), i32, vp, vp, vp]
        L.cb_apply_derivative.argtypes = [vp, ctypes.POINTER(StencilC), ctypes.POINTER(Grid), i32, vp, vp, vp]
        L.cb_batch_workspace_size.argtypes = [i32]
        L.cb_batch_workspace_size.restype = ctypes.c_size_t
        L.cb_batch_workspace_bytes.argtypes = [ctypes.POINTER(BatchItem), i32]
        L.cb_batch_workspace_bytes.restype = ctypes.c_size_t
        L.cb_solve_batched.argtypes = [ctypes.POINTER(BatchItem), i32, vp, ctypes.c_size_t, i32, vp]
        L.cb_batch_build.argtypes = [ctypes.POINTER(BatchItem), i32, vp, ctypes.c_size_t, vp]
        L.cb_batch_launch.argtypes = [vp, i32, vp]
        L.cb_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.cb_plan_get_schedule.argtypes = [vp, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)]
        L.cb_plan_get_array.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_double), i64, ctypes.POINTER(i64)]
        L.cb_last_error.restype = ctypes.c_char_p
        for f in ("cb_plan", "cb_plan_destroy", "cb_rhs_stencil", "cb_solve", "cb_solve_noalloc", "cb_copy_lines",
                  "cb_apply_derivative",
                  "cb_solve_batched", "cb_batch_build", "cb_batch_launch", "cb_plan_get_info",
                  "cb_plan_get_schedule", "cb_plan_get_array"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status):
    if status != CB_OK:
        raise CbError(status, lib().cb_last_error().decode())


class Stencil:
    """Periodic RHS stencil b_j = sum_{q=lo}^{lo+len-1} coefs[q-lo] f_{j+q}."""

    def __init__(self, lo, coefs):
        coefs = [float(c) for c in coefs]
        if not (-3 <= lo and lo + len(coefs) - 1 <= 3 and len(coefs) >= 1):
            raise ValueError("stencil must fit in offsets -3..3")
        self.lo, self.coefs = lo, coefs
        self.c = StencilC(lo, lo + len(coefs) - 1, (ctypes.c_double * 7)(*(coefs + [0.0] * (7 - len(coefs)))))


class Plan:
    """Pre-factorised compact banded matrix (cb_plan)."""

    def __init__(self, bands, n, cyclic=True, partitions=0, precision="fp64", refine_iters=0,
                 rows_per_lane=0, per_row=False, host_only=False, lines_per_wg=0, block_barriers=0,
                 x_staging=0, interior=0, tile_order=0):
        import numpy as np
        b = np.ascontiguousarray(np.asarray(bands, dtype=np.float64))
        r = (b.shape[-1] - 1) // 2
        self._bands = b
        d = PlanDesc(r, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(per_row), int(cyclic),
                     int(partitions), PRECISIONS[precision], int(refine_iters), int(rows_per_lane),
                     int(host_only), int(lines_per_wg), int(block_barriers), int(x_staging), int(interior),
                     int(tile_order))
        h = ctypes.c_void_p()
        _check(lib().cb_plan(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.n, self.r, self.precision, self.cyclic = n, r, precision, bool(cyclic)

    def close(self):
        if getattr(self, "h", None):
            lib().cb_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        i = PlanInfo()
        _check(lib().cb_plan_get_info(self.h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in PlanInfo._fields_}

    def schedule(self):
        """Detached rows per level of the workgroup-level reduced solve."""
        ln = ctypes.c_int32()
        _check(lib().cb_plan_get_schedule(self.h, None, 0, ctypes.byref(ln)))
        buf = (ctypes.c_int32 * max(ln.value, 1))()
        _check(lib().cb_plan_get_schedule(self.h, buf, ln.value, ctypes.byref(ln)))
        levels, cur = [], []
        for v in buf[:ln.value]:
            if v < 0:
                levels.append(cur)
                cur = []
            else:
                cur.append(v)
        return levels

    def array(self, which, seg=0):
        import numpy as np
        ln = ctypes.c_int64()
        _check(lib().cb_plan_get_array(self.h, seg, which, None, 0, ctypes.byref(ln)))
        out = np.zeros(max(ln.value, 1))
        _check(lib().cb_plan_get_array(self.h, seg, which, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       ln.value, ctypes.byref(ln)))
        return out[:ln.value]


def grid_of(t):
    """cb_grid of a 3D (nz, ny, nx) tensor (any positive strides)."""
    if t.dim() != 3:
        raise ValueError("expected a 3D (nz, ny, nx) tensor")
    g = Grid()
    g.n[0], g.n[1], g.n[2] = t.shape[2], t.shape[1], t.shape[0]
    st = t.stride()
    g.stride[0], g.stride[1], g.stride[2] = st[2], st[1], st[0]
    return g


def _dev(t):
    if not (t.is_cuda and t.dtype == torch.float64):
        raise ValueError("expected a float64 tensor on a ROCm device")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def solve(plan, b, axis, out=None, stream=None):
    """x = A^{-1} b along axis (0 x, 1 y, 2 z) of a (nz, ny, nx) tensor."""
    if out is None:
        out = torch.empty_like(b)
    g = grid_of(b)
    if grid_of(out).stride[:] != g.stride[:]:
        raise ValueError("b and out must have the same layout")
    _check(lib().cb_solve(plan.h, ctypes.byref(g), axis, _dev(b), _dev(out), _stream(stream)))
    return out


def solve_noalloc(plan, b, axis, out, stream=None):
    """cb_solve_noalloc: as solve(), with the partition scratch in the
    library's fixed per-GPU array (no device allocation; `out` is required)."""
    g = grid_of(b)
    if grid_of(out).stride[:] != g.stride[:]:
        raise ValueError("b and out must have the same layout")
    _check(lib().cb_solve_noalloc(plan.h, ctypes.byref(g), axis, _dev(b), _dev(out), _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 32 << 20  # CB_NOALLOC_SCRATCH_BYTES


def copy_lines(plan, f, axis, out=None, stream=None):
    """cb_copy_lines: out = f moved with the plan's launch along `axis` and no
    arithmetic (the access pattern's ceiling, for the roofline)."""
    if out is None:
        out = torch.empty_like(f)
    g = grid_of(f)
    if grid_of(out).stride[:] != g.stride[:]:
        raise ValueError("f and out must have the same layout")
    _check(lib().cb_copy_lines(plan.h, ctypes.byref(g), axis, _dev(f), _dev(out), _stream(stream)))
    return out


def apply_derivative(plan, stencil, f, axis, out=None, stream=None):
    """out = A^{-1} stencil(f) along axis (fused compact derivative/interpolation)."""
    if out is None:
        out = torch.empty_like(f)
    g = grid_of(f)
    if grid_of(out).stride[:] != g.stride[:]:
        raise ValueError("f and out must have the same layout")
    _check(lib().cb_apply_derivative(plan.h, ctypes.byref(stencil.c), ctypes.byref(g), axis, _dev(f),
                                     _dev(out), _stream(stream)))
    return out


def rhs_stencil(stencil, f, axis, out=None, stream=None):
    """b = stencil(f) along axis (periodic)."""
    if out is None:
        out = torch.empty_like(f)
    g = grid_of(f)
    if grid_of(out).stride[:] != g.stride[:]:
        raise ValueError("f and out must have the same layout")
    _check(lib().cb_rhs_stencil(ctypes.byref(stencil.c), ctypes.byref(g), axis, _dev(f), _dev(out),
                                _stream(stream)))
    return out


def batch_items(items):
    """ctypes cb_batch_item array of (plan, stencil or None, f, out, axis) tuples."""
    arr = (BatchItem * len(items))()
    for i, (plan, st, f, out, axis) in enumerate(items):
        g = grid_of(f)
        if grid_of(out).stride[:] != g.stride[:]:
            raise ValueError("f and out must have the same layout")
        arr[i].plan = plan.h
        arr[i].stencil = ctypes.pointer(st.c) if st is not None else None
        arr[i].grid = g
        arr[i].axis = axis
        arr[i].inp = _dev(f).value
        arr[i].out = _dev(out).value
    return arr


class Batch:
    """A built batched launch (cb_batch_build) over (plan, stencil or None, f,
    out, axis) items, with its device workspace sized by
    cb_batch_workspace_bytes.  launch() runs every item (cb_batch_launch);
    the plans, stencils and tensors must outlive the batch."""

    def __init__(self, items, stream=None, workspace=None):
        """`workspace`: a uint8 device tensor to build in when it is large
        enough (a rebuilt batch may reuse its predecessor's once that one's
        launches have finished), else a new one is allocated."""
        self.items = list(items)  # keeps plans, stencils and tensors alive
        arr = batch_items(self.items)
        need = lib().cb_batch_workspace_bytes(arr, len(self.items))
        if workspace is not None and workspace.numel() >= need:
            self.ws = workspace
        else:
            self.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.items[0][2].device)
        _check(lib().cb_batch_build(arr, len(self.items), ctypes.c_void_p(self.ws.data_ptr()), need,
                                    _stream(stream)))

    def launch(self, max_ctas=-1, stream=None):
        """max_ctas -1: one workgroup per tile; 0: persistent, one resident grid;
        > 0: persistent with at most that many workgroups."""
        _check(lib().cb_batch_launch(ctypes.c_void_p(self.ws.data_ptr()), int(max_ctas), _stream(stream)))
