"""MI355X-native fused sparse executor (Python binding of libsparsefusion.so).

Runs two sparse kernels, at least one with loop-carried dependences, as one
schedule over their joint dependence DAG (Cheshmi, Strout, Mehri Dehnavi,
"Composing Loop-carried Dependence with Other Loops", arXiv 2111.12238):
SpTRSV -> SpMV and SpIC0 -> SpTRSV, plus the adjoint of y = A L^{-1} b,
batched right-hand sides and FP32 solves with FP64 refinement.

This module only marshals arguments: every step of the computation runs in
the HIP kernels of ``libsparsefusion.so`` (see ``include/sf.h`` for the
C ABI).  PyTorch supplies device memory and the current stream.  If the
library is missing the import of any executor fails loudly; there is no
CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsparsefusion.so")

SF_F64, SF_F32 = 0, 1
SF_TRSV_SPMV, SF_IC0_TRSV, SF_ILU0_TRSV = 0, 1, 2
SF_STATIC_MSP, SF_STATIC_WAVEFRONT = 0, 1

STATUS = {
    0: "SF_OK", 1: "SF_ERR_ARG", 2: "SF_ERR_CSR", 3: "SF_ERR_NOT_LOWER", 4: "SF_ERR_ZERO_DIAG",
    5: "SF_ERR_SHAPE", 6: "SF_ERR_NOT_SPD", 7: "SF_ERR_HIP", 8: "SF_ERR_OOM", 9: "SF_ERR_TIMEOUT",
    10: "SF_ERR_UNSUPPORTED",
}


class SparseFusionError(RuntimeError):
    """A libsparsefusion call returned a status other than SF_OK."""

    def __init__(self, status: int, where: str, row: Optional[int] = None):
        self.status = int(status)
        self.name = STATUS.get(self.status, "SF_ERR_%d" % status)
        self.row = row
        msg = "%s: %s (%s)" % (where, self.name, _lib().sf_status_str(self.status).decode())
        if row is not None:
            msg += " at row %d" % row
        super().__init__(msg)


class CsrPattern(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int32), ("ncols", ctypes.c_int32),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p)]


class InspectOpts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in
                ("kind", "rows_per_item", "max_item_nnz", "rhs_block", "lanes_per_row",
                 "want_backward", "validate", "no_fusion", "coarsen")]


SF_PROBE_COPY, SF_PROBE_HOP, SF_PROBE_GATHER = 1, 2, 4


class ProbeResult(ctypes.Structure):
    _fields_ = [("copy_GBps", ctypes.c_double), ("hop_us_same_xcd", ctypes.c_double),
                ("hop_us_cross_xcd", ctypes.c_double), ("gathers_per_s", ctypes.c_double)]


class ScheduleStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("nnz_l", ctypes.c_int64),
                ("nnz_a", ctypes.c_int64), ("depth", ctypes.c_int32), ("joint_depth", ctypes.c_int32),
                ("back_depth", ctypes.c_int32), ("n_items", ctypes.c_int32),
                ("n_back_items", ctypes.c_int32), ("max_level_width", ctypes.c_int32),
                ("lanes_per_row", ctypes.c_int32), ("lanes_per_spmv", ctypes.c_int32),
                ("reuse_ratio", ctypes.c_double), ("inspect_seconds", ctypes.c_double),
                ("coarsened", ctypes.c_int32), ("chunk_items", ctypes.c_int32),
                ("chunk_chain", ctypes.c_int32), ("max_local_depth", ctypes.c_int32),
                ("est_level_us", ctypes.c_double), ("est_chunk_us", ctypes.c_double),
                ("back_coarsened", ctypes.c_int32), ("back_chunk_chain", ctypes.c_int32),
                ("est_back_level_us", ctypes.c_double), ("est_back_chunk_us", ctypes.c_double)]


_LIB = None
_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "sf_inspect": [ctypes.POINTER(CsrPattern), ctypes.POINTER(CsrPattern), ctypes.POINTER(InspectOpts),
                   ctypes.POINTER(_P)],
    "sf_schedule_free": [_P],
    "sf_schedule_info": [_P, ctypes.POINTER(ScheduleStats)],
    "sf_schedule_export": [_P, _P, _P, _P],
    "sf_schedule_export_local": [_P, _P, _P],
    "sf_schedule_export_backward_local": [_P, _P, _P],
    "sf_schedule_export_backward": [_P, _P, _P, _P],
    "sf_exec_trsv_spmv": [_P, _I, _P, _P, _P, _I, _I, _P, _I, _P, _I, _P],
    "sf_exec_unfused_trsv_spmv": [_P, _I, _P, _P, _P, _I, _I, _P, _I, _P, _I, _P],
    "sf_schedule_static_info": [_P, _I, _P, _P, _P, _P, _P],
    "sf_schedule_export_static": [_P, _I, _P, _P, _P],
    "sf_exec_static_trsv_spmv": [_P, _I, _I, _P, _P, _P, _P, _P, _P],
    "sf_exec_ic0_trsv": [_P, _I, _P, _P, _P, _I, _I, _P, _I, _P, _P],
    "sf_exec_unfused_ic0_trsv": [_P, _I, _P, _P, _P, _I, _I, _P, _I, _P, _P],
    "sf_backward": [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
    "sf_backward_noalloc": [_P, _I, _P, _P, _P, _P, _P, _P, _P, _P],
    "sf_refine_trsv_spmv": [_P, _P, _P, _P, _P, _I, _I, _P, _I, _P, _I, _I, _P, _P, ctypes.c_size_t, _P],
    "sf_set_param": [_P, ctypes.c_char_p, ctypes.c_int64],
    "sf_get_param": [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)],
    "sf_autotune": [_P, _I, _P, _P, _P, _I, _I, _P, _I, _P, _I, _P, ctypes.POINTER(ctypes.c_double)],
    "sf_sync_status": [_P, _P],
    "sf_last_kernel_ms": [_P, ctypes.POINTER(ctypes.c_double)],
    "sf_device_probe": [_I, _P, _P],
    "sf_trace_export": [_P, _P, ctypes.c_int64],
    "sf_exec_spmv_trsv": [_P, _I, _P, _P, _P, _P, _P, _P],
    "sf_exec_unfused_spmv_trsv": [_P, _I, _P, _P, _P, _P, _P, _P],
    "sf_exec_trsv_trsv": [_P, _I, _P, _P, _P, _P, _P],
    "sf_exec_unfused_trsv_trsv": [_P, _I, _P, _P, _P, _P, _P],
    "sf_exec_ic_apply": [_P, _I, _P, _P, _P, _P, _P],
    "sf_exec_ilu0_trsv": [_P, _I, _P, _P, _P, _P, _P, _P],
    "sf_exec_unfused_ilu0_trsv": [_P, _I, _P, _P, _P, _P, _P, _P],
    "sf_exec_unfused_ic_apply": [_P, _I, _P, _P, _P, _P, _P],
}


def _lib():
    """Load libsparsefusion.so (built by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsparsefusion.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.sf_status_str.argtypes = [ctypes.c_int]
        lib.sf_status_str.restype = ctypes.c_char_p
        lib.sf_version.restype = ctypes.c_char_p
        lib.sf_backward_workspace_bytes.argtypes = [_P, _I, _I]
        lib.sf_backward_workspace_bytes.restype = ctypes.c_size_t
        lib.sf_refine_workspace_bytes.argtypes = [_P, _I]
        lib.sf_refine_workspace_bytes.restype = ctypes.c_size_t
        _LIB = lib
    return _LIB


def _check(st, where, row=None):
    if st != 0:
        raise SparseFusionError(st, where, row)


def _pattern(rowptr, col, ncols):
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, np.int32)
    p = CsrPattern(len(rp) - 1, int(ncols), rp.ctypes.data, ci.ctypes.data)
    return p, (rp, ci)


def _csr_parts(m):
    """Accept a synth.CSR-like object (rowptr, col, nrows, ncols), a scipy
    CSR matrix, a torch sparse CSR tensor, or a (rowptr, col, ncols) tuple.
    Column indices must be sorted within each row (sf_inspect checks)."""
    if hasattr(m, "rowptr"):
        return m.rowptr, m.col, m.ncols
    if hasattr(m, "indptr"):
        return m.indptr, m.indices, m.shape[1]
    if hasattr(m, "crow_indices"):
        return m.crow_indices().cpu().numpy(), m.col_indices().cpu().numpy(), m.shape[1]
    rp, ci, ncols = m
    return rp, ci, ncols


# Every schedule not yet freed.  At interpreter exit they are released by an
# atexit hook, which runs before torch and the HIP runtime are torn down; a
# schedule collected later (during finalisation) makes no device call.
_LIVE = weakref.WeakSet()


@atexit.register
def _free_live_schedules():
    for sch in list(_LIVE):
        try:
            sch.free()
        except Exception:
            pass


class Schedule:
    """Host-built schedule (``sf_inspect``); lives until ``free()`` or GC."""

    def __init__(self, L, A=None, kind: int = SF_TRSV_SPMV, *, rows_per_item=0, max_item_nnz=0,
                 rhs_block=0, lanes_per_row=0, want_backward=False, validate=False, no_fusion=False,
                 coarsen=0):
        lib = _lib()
        lrp, lci, lnc = _csr_parts(L)
        pl, keep_l = _pattern(lrp, lci, lnc)
        pa_ptr = None
        keep_a = None
        if A is not None:
            arp, aci, anc = _csr_parts(A)
            pa, keep_a = _pattern(arp, aci, anc)
            pa_ptr = ctypes.byref(pa)
        opts = InspectOpts(kind, rows_per_item, max_item_nnz, rhs_block, lanes_per_row,
                           int(want_backward), int(validate), int(no_fusion), int(coarsen))
        h = _P()
        _check(lib.sf_inspect(ctypes.byref(pl), pa_ptr, ctypes.byref(opts), ctypes.byref(h)), "sf_inspect")
        del keep_l, keep_a
        self._h = h
        self.kind = kind
        _LIVE.add(self)
        st = self.info()
        self.n, self.m = int(st.n), int(st.m)
        self.nnz_l, self.nnz_a = int(st.nnz_l), int(st.nnz_a)

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise ValueError("schedule was freed")
        return self._h

    def info(self) -> ScheduleStats:
        st = ScheduleStats()
        _check(_lib().sf_schedule_info(self.handle, ctypes.byref(st)), "sf_schedule_info")
        return st

    def export(self):
        """(level[n], order[ids], item_ptr[n_items + 1]) as numpy arrays."""
        st = self.info()
        n = int(st.n)
        nids = n + int(st.m) if self.kind == SF_TRSV_SPMV else 2 * n
        level = np.empty(max(n, 1), np.int32)
        order = np.empty(max(nids, 1), np.int32)
        item_ptr = np.empty(int(st.n_items) + 1, np.int32)
        _check(_lib().sf_schedule_export(self.handle, level.ctypes.data, order.ctypes.data,
                                         item_ptr.ctypes.data), "sf_schedule_export")
        return level[:n], order[:nids], item_ptr

    def static_info(self, plan: int) -> dict:
        """Sizes of a static plan (SF_STATIC_MSP or SF_STATIC_WAVEFRONT)."""
        v = [ctypes.c_int32() for _ in range(5)]
        _check(_lib().sf_schedule_static_info(self.handle, plan, *[ctypes.byref(x) for x in v]),
               "sf_schedule_static_info")
        keys = ("n_spart", "n_wpart", "n_batches", "merged", "slack_moved")
        return {k: int(x.value) for k, x in zip(keys, v)}

    def export_static(self, plan: int):
        """(s_ptr, w_ptr, order) of a static plan as numpy arrays."""
        inf = self.static_info(plan)
        s_ptr = np.empty(inf["n_spart"] + 1, np.int32)
        w_ptr = np.empty(inf["n_wpart"] + 1, np.int32)
        order = np.empty(max(self.n + self.m, 1), np.int32)
        _check(_lib().sf_schedule_export_static(self.handle, plan, s_ptr.ctypes.data, w_ptr.ctypes.data,
                                                order.ctypes.data), "sf_schedule_export_static")
        return s_ptr, w_ptr, order[:self.n + self.m]

    def export_local(self):
        """(local_level[ids], entry_slot[nnz(L)]) of the exported plan: each
        claim position's wavefront inside its item, and per stored L entry the
        slot of its column in the row's item (255: another item)."""
        st = self.info()
        n = int(st.n)
        nids = n + int(st.m) if self.kind == SF_TRSV_SPMV else 2 * n
        loc = np.empty(max(nids, 1), np.uint8)
        slot = np.empty(max(int(st.nnz_l), 1), np.uint8)
        _check(_lib().sf_schedule_export_local(self.handle, loc.ctypes.data, slot.ctypes.data),
               "sf_schedule_export_local")
        return loc[:nids], slot[:int(st.nnz_l)]

    def export_backward_local(self):
        """(local_level[n], entry_slot[nnz(L)]) of the backward plan; entry
        slots are in the CSR order of L^T."""
        st = self.info()
        n = int(st.n)
        loc = np.empty(max(n, 1), np.uint8)
        slot = np.empty(max(int(st.nnz_l), 1), np.uint8)
        _check(_lib().sf_schedule_export_backward_local(self.handle, loc.ctypes.data, slot.ctypes.data),
               "sf_schedule_export_backward_local")
        return loc[:n], slot[:int(st.nnz_l)]

    def export_backward(self):
        st = self.info()
        n = int(st.n)
        rl = np.empty(max(n, 1), np.int32)
        order = np.empty(max(n, 1), np.int32)
        item_ptr = np.empty(int(st.n_back_items) + 1, np.int32)
        _check(_lib().sf_schedule_export_backward(self.handle, rl.ctypes.data, order.ctypes.data,
                                                  item_ptr.ctypes.data), "sf_schedule_export_backward")
        return rl[:n], order[:n], item_ptr

    def set_param(self, key: str, value: int):
        _check(_lib().sf_set_param(self.handle, key.encode(), int(value)), "sf_set_param(%s)" % key)

    def get_param(self, key: str) -> int:
        v = ctypes.c_int64()
        _check(_lib().sf_get_param(self.handle, key.encode(), ctypes.byref(v)), "sf_get_param(%s)" % key)
        return int(v.value)

    def last_kernel_ms(self) -> float:
        v = ctypes.c_double()
        _check(_lib().sf_last_kernel_ms(self.handle, ctypes.byref(v)), "sf_last_kernel_ms")
        return float(v.value)

    def trace(self):
        """Trace of the last traced fused single-RHS launch (needs
        set_param("trace", 1)): items (n_items, 8) -- real-time-counter
        stamps (100 MHz) at start, loads issued, inputs ready and end, then
        the run count -- and iterations (n + m, 2): the stamp taken just
        before each iteration's value was published and its publication
        count (ids as in export(): SpTRSV row i, SpMV row n + r)."""
        n_items = int(self.info().n_items)
        nids = self.n + self.m
        out = np.zeros(8 * n_items + 2 * nids, np.uint64)
        _check(_lib().sf_trace_export(self.handle, out.ctypes.data, out.size), "sf_trace_export")
        return out[:8 * n_items].reshape(n_items, 8), out[8 * n_items:].reshape(nids, 2)

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().sf_schedule_free(self._h)
        self._h = None
        _LIVE.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # during interpreter shutdown the HIP runtime may already be gone:
        # the atexit hook has released every schedule that was still live
        # (module globals may be cleared by now, hence the bound default)
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------- executors ----
def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return SF_F64
    if t.dtype == torch.float32:
        return SF_F32
    raise TypeError("values must be float64 or float32, got %s" % t.dtype)


def _vec_ptr(t, rows, name, dtype=None, device=None):
    """Device pointer, leading dimension and column count of a 1-D (n) or
    column-major 2-D (n, k) device tensor: unit stride down each column and
    columns that do not overlap.  dtype / device, when given, must match."""
    if t is None:
        raise ValueError("%s is required" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s: dtype %s, expected %s" % (name, t.dtype, dtype))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if t.dim() == 1:
        if t.shape[0] != rows or (rows > 1 and t.stride(0) != 1):
            raise ValueError("%s: expected a contiguous vector of length %d" % (name, rows))
        ld, k = max(rows, 1), 1
    elif t.dim() == 2 and t.shape[0] == rows:
        if rows > 1 and t.stride(0) != 1:
            raise ValueError("%s: rows must be contiguous (stride(0) = %d, expected 1)" % (name, t.stride(0)))
        if t.shape[1] > 1 and t.stride(1) < rows:
            raise ValueError("%s: columns overlap (stride %d < %d rows)" % (name, t.stride(1), rows))
        ld, k = (t.stride(1) if t.shape[1] > 1 else max(rows, 1)), t.shape[1]
    else:
        raise ValueError("%s: expected shape (%d,) or column-major (%d, k)" % (name, rows, rows))
    if device is None and not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    return t.data_ptr(), max(ld, 1), k


def _val_ptr(t, count, name, dtype, device):
    """Device pointer of a contiguous array of `count` matrix values in the
    CSR order of the inspected pattern (None allowed only when count == 0)."""
    if t is None:
        if count == 0:
            return None
        raise ValueError("%s is required (%d stored entries)" % (name, count))
    if t.dtype != dtype:
        raise ValueError("%s: dtype %s, expected %s" % (name, t.dtype, dtype))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    if t.numel() != count:
        raise ValueError("%s has %d values, the pattern stores %d" % (name, t.numel(), count))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _gpu(device):
    """Every tensor of a call was checked to sit on `device`: it must be a GPU."""
    if device is None or device.type != "cuda":
        raise ValueError("the tensors must be on a GPU device, not %s" % device)


def _float_dtype(t, name):
    torch = _torch()
    if t is None or not hasattr(t, "dtype"):
        raise ValueError("%s is required" % name)
    if t.dtype not in (torch.float64, torch.float32):
        raise TypeError("%s must be float64 or float32, got %s" % (name, t.dtype))
    return t.dtype


def colmajor(n, k, dtype, device="cuda"):
    """An uninitialised column-major (n, k) tensor (k == 1 gives a vector)."""
    torch = _torch()
    if k == 1:
        return torch.empty(n, dtype=dtype, device=device)
    return torch.empty((k, n), dtype=dtype, device=device).t()


def _ptr(t):
    return None if t is None else t.data_ptr()


def trsv_spmv(sched: Schedule, L_val, A_val, B, *, X=None, Y=None, want_y=True, stream=None,
              unfused=False):
    """x = L^{-1} b, y = A x (fused unless ``unfused``).  B: (n,) or (n, k).
    L_val, A_val, B, X and Y share one dtype (float64 or float32) and device."""
    n, m = sched.n, sched.m
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    ap = _val_ptr(A_val, sched.nnz_a, "A_val", dt, dev) if want_y else None
    bp, ldb, k = _vec_ptr(B, n, "B", dt, dev)
    if X is None:
        X = colmajor(n, k, dt, dev)
    if want_y and Y is None:
        Y = colmajor(m, k, dt, dev)
    xp, ldx, kx = _vec_ptr(X, n, "X", dt, dev)
    yp, ldy, ky = (None, max(m, 1), k)
    if want_y:
        yp, ldy, ky = _vec_ptr(Y, m, "Y", dt, dev)
    if kx != k or ky != k:
        raise ValueError("B, X and Y must have the same number of columns (%d, %d, %d)" % (k, kx, ky))
    _gpu(dev)
    fn = _lib().sf_exec_unfused_trsv_spmv if unfused else _lib().sf_exec_trsv_spmv
    _check(fn(sched.handle, _dtype_code(L_val), lp, ap, bp, ldb, k, xp, ldx, yp, ldy,
              _stream(stream)), "sf_exec_trsv_spmv")
    return X, (Y if want_y else None)


def static_trsv_spmv(sched: Schedule, plan: int, L_val, A_val, b, *, X=None, Y=None, stream=None):
    """x = L^{-1} b, y = A x (one right-hand side) under a static plan:
    SF_STATIC_MSP (the paper's fused partitioning) or SF_STATIC_WAVEFRONT."""
    n, m = sched.n, sched.m
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    ap = _val_ptr(A_val, sched.nnz_a, "A_val", dt, dev)
    bp, _, k = _vec_ptr(b, n, "b", dt, dev)
    if k != 1:
        raise ValueError("static plans take one right-hand side")
    if X is None:
        X = colmajor(n, 1, dt, dev)
    if Y is None and m > 0:
        Y = colmajor(m, 1, dt, dev)
    xp, _, kx = _vec_ptr(X, n, "X", dt, dev)
    yp = _vec_ptr(Y, m, "Y", dt, dev)[0] if m > 0 else None
    if kx != 1 or (m > 0 and Y.numel() != m):
        raise ValueError("X and Y must be single vectors")
    _gpu(dev)
    _check(_lib().sf_exec_static_trsv_spmv(sched.handle, plan, _dtype_code(L_val), lp, ap, bp, xp, yp,
                                           _stream(stream)), "sf_exec_static_trsv_spmv")
    return X, Y


def _one_vec(t, n, name, dt, dev):
    p, _, k = _vec_ptr(t, n, name, dt, dev)
    if k != 1:
        raise ValueError("%s: one right-hand side expected" % name)
    return p


def spmv_trsv(sched: Schedule, A_val, L_val, x, *, Y=None, Z=None, want_y=True, stream=None, unfused=False):
    """y = A x, z = L^{-1} y (Table 2, combination 2).  Returns (y or None, z)."""
    n = sched.n
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    ap = _val_ptr(A_val, sched.nnz_a, "A_val", dt, dev)
    xp = _one_vec(x, n, "x", dt, dev)
    torch = _torch()
    if Z is None:
        Z = torch.empty(n, dtype=dt, device=dev)
    if (want_y or unfused) and Y is None:
        Y = torch.empty(n, dtype=dt, device=dev)
    yp = _one_vec(Y, n, "Y", dt, dev) if (want_y or unfused) else None
    _gpu(dev)
    fn = _lib().sf_exec_unfused_spmv_trsv if unfused else _lib().sf_exec_spmv_trsv
    _check(fn(sched.handle, _dtype_code(L_val), ap, lp, xp, yp, _one_vec(Z, n, "Z", dt, dev),
              _stream(stream)), "sf_exec_spmv_trsv")
    return (Y if (want_y or unfused) else None), Z


def trsv_trsv(sched: Schedule, L_val, b, *, X=None, Z=None, stream=None, unfused=False):
    """x = L^{-1} b, z = L^{-1} x (Table 2, combination 1).  Returns (x, z)."""
    n = sched.n
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    bp = _one_vec(b, n, "b", dt, dev)
    torch = _torch()
    X = torch.empty(n, dtype=dt, device=dev) if X is None else X
    Z = torch.empty(n, dtype=dt, device=dev) if Z is None else Z
    _gpu(dev)
    fn = _lib().sf_exec_unfused_trsv_trsv if unfused else _lib().sf_exec_trsv_trsv
    _check(fn(sched.handle, _dtype_code(L_val), lp, bp, _one_vec(X, n, "X", dt, dev),
              _one_vec(Z, n, "Z", dt, dev), _stream(stream)), "sf_exec_trsv_trsv")
    return X, Z


def ic_apply(sched: Schedule, L_val, r, *, W=None, Z=None, stream=None, unfused=False):
    """w = L^{-1} r, z = L^{-T} w (the incomplete-Cholesky preconditioner
    apply); the schedule needs want_backward=True.  Returns (w, z)."""
    n = sched.n
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    rp = _one_vec(r, n, "r", dt, dev)
    torch = _torch()
    W = torch.empty(n, dtype=dt, device=dev) if W is None else W
    Z = torch.empty(n, dtype=dt, device=dev) if Z is None else Z
    _gpu(dev)
    fn = _lib().sf_exec_unfused_ic_apply if unfused else _lib().sf_exec_ic_apply
    _check(fn(sched.handle, _dtype_code(L_val), lp, rp, _one_vec(W, n, "W", dt, dev),
              _one_vec(Z, n, "Z", dt, dev), _stream(stream)), "sf_exec_ic_apply")
    return W, Z


def ilu0_trsv(sched: Schedule, A_val, x=None, *, LU_val=None, Y=None, stream=None, unfused=False,
              check_info=True):
    """L U ~= A (zero fill, Table 2 combination 6) and y = L^{-1} x in one
    launch (float64).  Returns (LU values in A's pattern, y or None, info)."""
    torch = _torch()
    n = sched.n
    f64 = torch.float64
    dev = A_val.device if hasattr(A_val, "device") else None
    ap = _val_ptr(A_val, sched.nnz_l, "A_val", f64, dev)
    LU_val = torch.empty_like(A_val) if LU_val is None else LU_val
    lup = _val_ptr(LU_val, sched.nnz_l, "LU_val", f64, dev)
    info = torch.full((1,), -1, dtype=torch.int32, device=dev)
    xp = yp = None
    if x is not None:
        xp = _one_vec(x, n, "x", f64, dev)
        Y = torch.empty(n, dtype=f64, device=dev) if Y is None else Y
        yp = _one_vec(Y, n, "Y", f64, dev)
    _gpu(dev)
    fn = _lib().sf_exec_unfused_ilu0_trsv if unfused else _lib().sf_exec_ilu0_trsv
    _check(fn(sched.handle, SF_F64, ap, lup, xp, yp, info.data_ptr(), _stream(stream)), "sf_exec_ilu0_trsv")
    if check_info:
        row = int(info.item())
        if row >= 0:
            raise SparseFusionError(6, "sf_exec_ilu0_trsv", row)
    return LU_val, (Y if x is not None else None), info


def ic0_trsv(sched: Schedule, A_lower_val, b=None, *, L_val=None, X=None, stream=None, unfused=False,
             check_info=True):
    """L L^T ~= A (zero fill) and x = L^{-1} b in one launch (float64).
    Returns (L_val, x, info)."""
    torch = _torch()
    n = sched.n
    f64 = torch.float64
    dev = A_lower_val.device if hasattr(A_lower_val, "device") else None
    ap = _val_ptr(A_lower_val, sched.nnz_l, "A_lower_val", f64, dev)
    if L_val is None:
        L_val = torch.empty_like(A_lower_val)
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", f64, dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    bp, ldb = None, max(n, 1)
    xp, ldx = None, max(n, 1)
    if b is not None:
        bp, ldb, kb = _vec_ptr(b, n, "b", f64, dev)
        if X is None:
            X = torch.empty(n, dtype=f64, device=dev)
        xp, ldx, kx = _vec_ptr(X, n, "X", f64, dev)
        if kb != 1 or kx != 1:
            raise ValueError("ic0_trsv takes one right-hand side")
    _gpu(dev)
    fn = _lib().sf_exec_unfused_ic0_trsv if unfused else _lib().sf_exec_ic0_trsv
    _check(fn(sched.handle, SF_F64, ap, lp, bp, ldb, 1, xp, ldx, info.data_ptr(), _stream(stream)),
           "sf_exec_ic0_trsv")
    row = None
    if check_info:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        row = int(info.item())
        if row >= 0:
            raise SparseFusionError(6, "sf_exec_ic0_trsv", row)
    return L_val, X, info


def backward(sched: Schedule, L_val, A_val, G, *, X=None, B=None, stream=None):
    """(grad_b, grad_L_val) of loss with dloss/dy = G; X or B (recompute) needed.
    Every tensor shares L_val's dtype and device."""
    torch = _torch()
    n, m = sched.n, sched.m
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    ap = _val_ptr(A_val, sched.nnz_a, "A_val", dt, dev)
    gp = _one_vec(G, m, "G", dt, dev)
    xp = _one_vec(X, n, "X", dt, dev) if X is not None else None
    bp = _one_vec(B, n, "B", dt, dev) if B is not None else None
    if xp is None and bp is None:
        raise ValueError("backward needs X (stored) or B (recompute x)")
    grad_b = torch.empty(n, dtype=dt, device=dev)
    grad_l = torch.empty_like(L_val)
    ws, wsb = None, 0
    if X is None:
        wsb = int(_lib().sf_backward_workspace_bytes(sched.handle, _dtype_code(L_val), 1))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    _gpu(dev)
    _check(_lib().sf_backward(sched.handle, _dtype_code(L_val), lp, ap, xp, bp, gp, grad_b.data_ptr(),
                              grad_l.data_ptr(), _ptr(ws), wsb, _stream(stream)), "sf_backward")
    return grad_b, grad_l


def refine_trsv_spmv(sched: Schedule, L32, L64, A64, B, *, n_corrections=2, want_y=True, stream=None):
    """FP32 fused solves + FP64 residual refinement.  L32 float32; L64, A64
    and B float64, all on one device.  Returns (X, Y, relres)."""
    torch = _torch()
    n, m = sched.n, sched.m
    dev = B.device
    l32 = _val_ptr(L32, sched.nnz_l, "L32", torch.float32, dev)
    l64 = _val_ptr(L64, sched.nnz_l, "L64", torch.float64, dev)
    a64 = _val_ptr(A64, sched.nnz_a, "A64", torch.float64, dev) if want_y else None
    bp, ldb, k = _vec_ptr(B, n, "B", torch.float64, dev)
    X = colmajor(n, k, torch.float64, dev)
    xp, ldx, _ = _vec_ptr(X, n, "X", torch.float64, dev)
    Y, yp, ldy = None, None, max(m, 1)
    if want_y:
        Y = colmajor(m, k, torch.float64, dev)
        yp, ldy, _ = _vec_ptr(Y, m, "Y", torch.float64, dev)
    wsb = int(_lib().sf_refine_workspace_bytes(sched.handle, k))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    rel = (ctypes.c_double * k)()
    _gpu(dev)
    _check(_lib().sf_refine_trsv_spmv(sched.handle, l32, l64, a64, bp, ldb, k, xp, ldx, yp, ldy,
                                      int(n_corrections), rel, ws.data_ptr(), wsb, _stream(stream)),
           "sf_refine_trsv_spmv")
    return X, Y, np.array(rel[:], dtype=np.float64)


def autotune(sched: Schedule, L_val, A_val, B, *, want_y=True, stream=None):
    """Time executor variants on the caller's data and keep the fastest."""
    n, m = sched.n, sched.m
    dt = _float_dtype(L_val, "L_val")
    dev = L_val.device
    lp = _val_ptr(L_val, sched.nnz_l, "L_val", dt, dev)
    ap = _val_ptr(A_val, sched.nnz_a, "A_val", dt, dev) if want_y else None
    bp, ldb, k = _vec_ptr(B, n, "B", dt, dev)
    X = colmajor(n, k, dt, dev)
    xp, ldx, _ = _vec_ptr(X, n, "X", dt, dev)
    yp, ldy = None, max(m, 1)
    if want_y:
        Y = colmajor(m, k, dt, dev)
        yp, ldy, _ = _vec_ptr(Y, m, "Y", dt, dev)
    best = ctypes.c_double()
    _gpu(dev)
    _check(_lib().sf_autotune(sched.handle, _dtype_code(L_val), lp, ap, bp, ldb, k,
                              xp, ldx, yp, ldy, _stream(stream), ctypes.byref(best)), "sf_autotune")
    return float(best.value)


def sync_status(sched: Schedule, stream=None):
    """Synchronise and raise SparseFusionError(SF_ERR_TIMEOUT) if a watchdog fired."""
    _check(_lib().sf_sync_status(sched.handle, _stream(stream)), "sf_sync_status")


def device_probe(what: int = 0, stream=None) -> dict:
    """Machine constants of the current device (``sf_device_probe``): copy
    ceiling (GB/s), one-way hop latency on one XCD and across XCDs (us), and
    random single-value gathers per second; -1 for what was not probed."""
    r = ProbeResult()
    _check(_lib().sf_device_probe(what, ctypes.byref(r), _stream(stream)), "sf_device_probe")
    return {k: getattr(r, k) for k, _ in ProbeResult._fields_}


def version() -> str:
    return _lib().sf_version().decode()


from .autograd import TrsvSpmv, trsv_spmv_autograd  # noqa: E402
