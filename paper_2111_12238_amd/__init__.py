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

import ctypes
import os
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
        """Per-item timestamps (n_items, 4) of the last traced fused launch, in
        100 MHz real-time-counter ticks (needs set_param("trace", 1))."""
        n_items = int(self.info().n_items)
        out = np.zeros(4 * max(n_items, 1), np.uint64)
        _check(_lib().sf_trace_export(self.handle, out.ctypes.data, out.size), "sf_trace_export")
        return out[:4 * n_items].reshape(n_items, 4)

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().sf_schedule_free(self._h)
        self._h = None

    def __del__(self):
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


def _vec_ptr(t, rows, name):
    """Device pointer and leading dimension of a 1-D (n) or column-major 2-D
    (n, k) CUDA tensor."""
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dim() == 1:
        if t.stride(0) != 1 or t.shape[0] != rows:
            raise ValueError("%s: expected a contiguous vector of length %d" % (name, rows))
        return t.data_ptr(), max(rows, 1), 1
    if t.dim() == 2 and t.shape[0] == rows and (t.stride(0) == 1 or t.shape[1] == 1):
        if t.shape[1] > 1 and t.stride(1) < rows:
            raise ValueError("%s: columns overlap (stride %d < %d rows)" % (name, t.stride(1), rows))
        ld = t.stride(1) if t.shape[1] > 1 else max(rows, 1)
        return t.data_ptr(), max(ld, 1), t.shape[1]
    raise ValueError("%s: expected shape (%d,) or column-major (%d, k)" % (name, rows, rows))


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
    """x = L^{-1} b, y = A x (fused unless ``unfused``).  B: (n,) or (n, k)."""
    n, m = sched.n, sched.m
    bp, ldb, k = _vec_ptr(B, n, "B")
    dt = _dtype_code(L_val)
    if X is None:
        X = colmajor(n, k, L_val.dtype, L_val.device)
    if want_y and Y is None:
        Y = colmajor(m, k, L_val.dtype, L_val.device)
    xp, ldx, _ = _vec_ptr(X, n, "X")
    yp, ldy = (None, max(m, 1))
    if want_y:
        yp, ldy, _ = _vec_ptr(Y, m, "Y")
    fn = _lib().sf_exec_unfused_trsv_spmv if unfused else _lib().sf_exec_trsv_spmv
    _check(fn(sched.handle, dt, L_val.data_ptr(), _ptr(A_val), bp, ldb, k, xp, ldx, yp, ldy,
              _stream(stream)), "sf_exec_trsv_spmv")
    return X, (Y if want_y else None)


def static_trsv_spmv(sched: Schedule, plan: int, L_val, A_val, b, *, X=None, Y=None, stream=None):
    """x = L^{-1} b, y = A x (one right-hand side) under a static plan:
    SF_STATIC_MSP (the paper's fused partitioning) or SF_STATIC_WAVEFRONT."""
    n, m = sched.n, sched.m
    bp, _, k = _vec_ptr(b, n, "b")
    if k != 1:
        raise ValueError("static plans take one right-hand side")
    if X is None:
        X = colmajor(n, 1, L_val.dtype, L_val.device)
    if Y is None and m > 0:
        Y = colmajor(m, 1, L_val.dtype, L_val.device)
    xp, _, _ = _vec_ptr(X, n, "X")
    yp = _vec_ptr(Y, m, "Y")[0] if m > 0 else None
    _check(_lib().sf_exec_static_trsv_spmv(sched.handle, plan, _dtype_code(L_val), L_val.data_ptr(),
                                           _ptr(A_val), bp, xp, yp, _stream(stream)), "sf_exec_static_trsv_spmv")
    return X, Y


def spmv_trsv(sched: Schedule, A_val, L_val, x, *, Y=None, Z=None, want_y=True, stream=None, unfused=False):
    """y = A x, z = L^{-1} y (Table 2, combination 2).  Returns (y or None, z)."""
    n = sched.n
    xp, _, k = _vec_ptr(x, n, "x")
    if k != 1:
        raise ValueError("spmv_trsv takes one right-hand side")
    torch = _torch()
    if Z is None:
        Z = torch.empty(n, dtype=L_val.dtype, device=L_val.device)
    if (want_y or unfused) and Y is None:
        Y = torch.empty(n, dtype=L_val.dtype, device=L_val.device)
    yp = _vec_ptr(Y, n, "Y")[0] if (want_y or unfused) else None
    fn = _lib().sf_exec_unfused_spmv_trsv if unfused else _lib().sf_exec_spmv_trsv
    _check(fn(sched.handle, _dtype_code(L_val), _ptr(A_val), L_val.data_ptr(), xp, yp, _vec_ptr(Z, n, "Z")[0],
              _stream(stream)), "sf_exec_spmv_trsv")
    return (Y if (want_y or unfused) else None), Z


def trsv_trsv(sched: Schedule, L_val, b, *, X=None, Z=None, stream=None, unfused=False):
    """x = L^{-1} b, z = L^{-1} x (Table 2, combination 1).  Returns (x, z)."""
    n = sched.n
    bp, _, k = _vec_ptr(b, n, "b")
    if k != 1:
        raise ValueError("trsv_trsv takes one right-hand side")
    torch = _torch()
    X = torch.empty(n, dtype=L_val.dtype, device=L_val.device) if X is None else X
    Z = torch.empty(n, dtype=L_val.dtype, device=L_val.device) if Z is None else Z
    fn = _lib().sf_exec_unfused_trsv_trsv if unfused else _lib().sf_exec_trsv_trsv
    _check(fn(sched.handle, _dtype_code(L_val), L_val.data_ptr(), bp, _vec_ptr(X, n, "X")[0],
              _vec_ptr(Z, n, "Z")[0], _stream(stream)), "sf_exec_trsv_trsv")
    return X, Z


def ic_apply(sched: Schedule, L_val, r, *, W=None, Z=None, stream=None, unfused=False):
    """w = L^{-1} r, z = L^{-T} w (the incomplete-Cholesky preconditioner
    apply); the schedule needs want_backward=True.  Returns (w, z)."""
    n = sched.n
    rp, _, k = _vec_ptr(r, n, "r")
    if k != 1:
        raise ValueError("ic_apply takes one right-hand side")
    torch = _torch()
    W = torch.empty(n, dtype=L_val.dtype, device=L_val.device) if W is None else W
    Z = torch.empty(n, dtype=L_val.dtype, device=L_val.device) if Z is None else Z
    fn = _lib().sf_exec_unfused_ic_apply if unfused else _lib().sf_exec_ic_apply
    _check(fn(sched.handle, _dtype_code(L_val), L_val.data_ptr(), rp, _vec_ptr(W, n, "W")[0],
              _vec_ptr(Z, n, "Z")[0], _stream(stream)), "sf_exec_ic_apply")
    return W, Z


def ilu0_trsv(sched: Schedule, A_val, x=None, *, LU_val=None, Y=None, stream=None, unfused=False,
              check_info=True):
    """L U ~= A (zero fill, Table 2 combination 6) and y = L^{-1} x in one
    launch.  Returns (LU values in A's pattern, y or None, info tensor)."""
    torch = _torch()
    n = sched.n
    LU_val = torch.empty_like(A_val) if LU_val is None else LU_val
    info = torch.full((1,), -1, dtype=torch.int32, device=A_val.device)
    xp = yp = None
    if x is not None:
        xp = _vec_ptr(x, n, "x")[0]
        Y = torch.empty(n, dtype=A_val.dtype, device=A_val.device) if Y is None else Y
        yp = _vec_ptr(Y, n, "Y")[0]
    fn = _lib().sf_exec_unfused_ilu0_trsv if unfused else _lib().sf_exec_ilu0_trsv
    _check(fn(sched.handle, _dtype_code(A_val), A_val.data_ptr(), LU_val.data_ptr(), xp, yp, info.data_ptr(),
              _stream(stream)), "sf_exec_ilu0_trsv")
    if check_info:
        row = int(info.item())
        if row >= 0:
            raise SparseFusionError(6, "sf_exec_ilu0_trsv", row)
    return LU_val, (Y if x is not None else None), info


def ic0_trsv(sched: Schedule, A_lower_val, b=None, *, L_val=None, X=None, stream=None, unfused=False,
             check_info=True):
    """L L^T ~= A (zero fill) and x = L^{-1} b in one launch.  Returns (L_val, x, info)."""
    torch = _torch()
    n = sched.n
    if L_val is None:
        L_val = torch.empty_like(A_lower_val)
    info = torch.empty(1, dtype=torch.int32, device=A_lower_val.device)
    bp, ldb = None, max(n, 1)
    xp, ldx = None, max(n, 1)
    if b is not None:
        bp, ldb, _ = _vec_ptr(b, n, "b")
        if X is None:
            X = torch.empty(n, dtype=torch.float64, device=b.device)
        xp, ldx, _ = _vec_ptr(X, n, "X")
    fn = _lib().sf_exec_unfused_ic0_trsv if unfused else _lib().sf_exec_ic0_trsv
    _check(fn(sched.handle, _dtype_code(A_lower_val), A_lower_val.data_ptr(), L_val.data_ptr(), bp, ldb, 1,
              xp, ldx, info.data_ptr(), _stream(stream)), "sf_exec_ic0_trsv")
    row = None
    if check_info:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        row = int(info.item())
        if row >= 0:
            raise SparseFusionError(6, "sf_exec_ic0_trsv", row)
    return L_val, X, info


def backward(sched: Schedule, L_val, A_val, G, *, X=None, B=None, stream=None):
    """(grad_b, grad_L_val) of loss with dloss/dy = G; X or B (recompute) needed."""
    torch = _torch()
    grad_b = torch.empty(sched.n, dtype=L_val.dtype, device=L_val.device)
    grad_l = torch.empty_like(L_val)
    ws, wsb = None, 0
    if X is None:
        wsb = int(_lib().sf_backward_workspace_bytes(sched.handle, _dtype_code(L_val), 1))
        ws = torch.empty(wsb, dtype=torch.uint8, device=L_val.device)
    _check(_lib().sf_backward(sched.handle, _dtype_code(L_val), L_val.data_ptr(), _ptr(A_val), _ptr(X),
                              _ptr(B), G.data_ptr(), grad_b.data_ptr(), grad_l.data_ptr(), _ptr(ws), wsb,
                              _stream(stream)), "sf_backward")
    return grad_b, grad_l


def refine_trsv_spmv(sched: Schedule, L32, L64, A64, B, *, n_corrections=2, want_y=True, stream=None):
    """FP32 fused solves + FP64 residual refinement.  Returns (X, Y, relres)."""
    torch = _torch()
    n, m = sched.n, sched.m
    bp, ldb, k = _vec_ptr(B, n, "B")
    X = colmajor(n, k, torch.float64, B.device)
    xp, ldx, _ = _vec_ptr(X, n, "X")
    Y, yp, ldy = None, None, max(m, 1)
    if want_y:
        Y = colmajor(m, k, torch.float64, B.device)
        yp, ldy, _ = _vec_ptr(Y, m, "Y")
    wsb = int(_lib().sf_refine_workspace_bytes(sched.handle, k))
    ws = torch.empty(wsb, dtype=torch.uint8, device=B.device)
    rel = (ctypes.c_double * k)()
    _check(_lib().sf_refine_trsv_spmv(sched.handle, L32.data_ptr(), L64.data_ptr(), _ptr(A64), bp, ldb, k,
                                      xp, ldx, yp, ldy, int(n_corrections), rel, ws.data_ptr(), wsb,
                                      _stream(stream)), "sf_refine_trsv_spmv")
    return X, Y, np.array(rel[:], dtype=np.float64)


def autotune(sched: Schedule, L_val, A_val, B, *, want_y=True, stream=None):
    """Time executor variants on the caller's data and keep the fastest."""
    n, m = sched.n, sched.m
    bp, ldb, k = _vec_ptr(B, n, "B")
    X = colmajor(n, k, L_val.dtype, L_val.device)
    xp, ldx, _ = _vec_ptr(X, n, "X")
    yp, ldy = None, max(m, 1)
    if want_y:
        Y = colmajor(m, k, L_val.dtype, L_val.device)
        yp, ldy, _ = _vec_ptr(Y, m, "Y")
    best = ctypes.c_double()
    _check(_lib().sf_autotune(sched.handle, _dtype_code(L_val), L_val.data_ptr(), _ptr(A_val), bp, ldb, k,
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
