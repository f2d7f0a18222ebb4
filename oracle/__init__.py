"""Sequential FP64 CPU oracle for the fused sparse executor.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it.  It shares no code with the HIP path; the arithmetic lives in
``sf_oracle.c`` (plain C, ``-ffp-contract=off``), and this module only
marshals numpy arrays into it.

Every function cites the passage of the paper (Cheshmi, Strout, Mehri
Dehnavi, arXiv 2111.12238) or the definition it follows; see the header of
``sf_oracle.c``.  All pins live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_c_int = ctypes.c_int


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    sig = {
        "orc_check_lower": (_c_int, [_c_int, _i32p, _i32p]),
        "orc_check_csr": (_c_int, [_c_int, _c_int, _i32p, _i32p]),
        "orc_trsv_lower": (None, [_c_int, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_spmv": (None, [_c_int, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_transpose": (None, [_c_int, _c_int, _i32p, _i32p, _i32p, _i32p, _i32p]),
        "orc_spmv_t": (None, [_c_int, _c_int, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_trsv_upper_t": (None, [_c_int, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_ic0": (_c_int, [_c_int, _i32p, _i32p, _f64p, _f64p]),
        "orc_ilu0": (_c_int, [_c_int, _i32p, _i32p, _f64p, _f64p]),
        "orc_trsv_unit_lower": (None, [_c_int, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_backward": (None, [_c_int, _c_int, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p,
                                _f64p, _f64p, _f64p, _f64p]),
        "orc_levels": (_c_int, [_c_int, _i32p, _i32p, _i32p]),
        "orc_reverse_levels": (_c_int, [_c_int, _i32p, _i32p, _i32p]),
        "orc_spmv_ready": (None, [_c_int, _i32p, _i32p, _i32p, _i32p]),
        "orc_joint_order_ts": (None, [_c_int, _i32p, _c_int, _i32p, _i32p]),
        "orc_validate_ts": (_c_int, [_c_int, _i32p, _i32p, _c_int, _i32p, _i32p, _i32p, _c_int,
                                     _i32p, _c_int]),
        "orc_validate_factor_solve": (_c_int, [_c_int, _i32p, _i32p, _i32p, _c_int, _i32p]),
        "orc_validate_static_ts": (_c_int, [_c_int, _i32p, _i32p, _c_int, _i32p, _i32p, _c_int, _i32p,
                                            _c_int, _i32p, _i32p]),
        "orc_reuse_ts": (ctypes.c_double, [_c_int, _c_int, _c_int, _c_int]),
        "orc_reuse_it": (ctypes.c_double, [_c_int, _c_int]),
        "orc_refine": (ctypes.c_double, [_c_int, _i32p, _i32p, _f64p, _f32p, _c_int, _i32p, _i32p, _f64p,
                                         _f64p, _c_int, _f64p, _f64p, ctypes.c_void_p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    # zero-length arrays still need a valid pointer for ctypes
    return a if a.size else np.zeros(1, dtype=a.dtype)


class Oracle:
    """The oracle's routines bound to one compiled copy of ``sf_oracle.c``."""

    def __init__(self, lib_path):
        self.lib = _bind(ctypes.CDLL(lib_path))

    def check_lower(self, rp, ci) -> int:
        """0 = valid lower CSR; 1 bad CSR; 2 entry above diagonal; 3 missing diagonal."""
        rp, ci = _i32(rp), _i32(ci)
        return self.lib.orc_check_lower(len(rp) - 1, rp, _ptr(ci))

    def check_csr(self, rp, ci, ncols) -> int:
        rp, ci = _i32(rp), _i32(ci)
        return self.lib.orc_check_csr(len(rp) - 1, ncols, rp, _ptr(ci))

    def trsv_lower(self, rp, ci, v, b):
        """x = L^{-1} b by forward substitution in row order (SpTRSV, Sec. 1)."""
        rp, ci, v, b = _i32(rp), _i32(ci), _f64(v), _f64(b)
        n = len(rp) - 1
        x = np.empty(n, np.float64)
        self.lib.orc_trsv_lower(n, rp, _ptr(ci), _ptr(v), _ptr(b), _ptr(x))
        return x

    def spmv(self, rp, ci, v, x):
        """y = A x, CSR, ascending nonzero order (SpMV, Sec. 1)."""
        rp, ci, v, x = _i32(rp), _i32(ci), _f64(v), _f64(x)
        m = len(rp) - 1
        y = np.empty(m, np.float64)
        self.lib.orc_spmv(m, rp, _ptr(ci), _ptr(v), _ptr(x), _ptr(y))
        return y

    def transpose(self, rp, ci, ncols):
        """CSR transpose: returns (trp, tci, perm) with perm mapping entries back."""
        rp, ci = _i32(rp), _i32(ci)
        m = len(rp) - 1
        nnz = int(rp[-1])
        trp = np.empty(ncols + 1, np.int32)
        tci = np.empty(nnz, np.int32)
        perm = np.empty(nnz, np.int32)
        self.lib.orc_transpose(m, ncols, rp, _ptr(ci), trp, _ptr(tci), _ptr(perm))
        return trp, tci, perm

    def spmv_t(self, rp, ci, v, g, ncols):
        """c = A^T g."""
        rp, ci, v, g = _i32(rp), _i32(ci), _f64(v), _f64(g)
        m = len(rp) - 1
        c = np.empty(ncols, np.float64)
        self.lib.orc_spmv_t(m, ncols, rp, _ptr(ci), _ptr(v), _ptr(g), _ptr(c))
        return c

    def trsv_upper_t(self, rp, ci, v, c):
        """lam = L^{-T} c by backward substitution."""
        rp, ci, v, c = _i32(rp), _i32(ci), _f64(v), _f64(c)
        n = len(rp) - 1
        lam = np.empty(n, np.float64)
        self.lib.orc_trsv_upper_t(n, rp, _ptr(ci), _ptr(v), _ptr(c), _ptr(lam))
        return lam

    def ic0(self, rp, ci, a_lower):
        """Zero fill-in incomplete Cholesky of lower(A) (Table 2, combination 5).

        Returns (L values in the same pattern, first failing row or -1)."""
        rp, ci, a = _i32(rp), _i32(ci), _f64(a_lower)
        n = len(rp) - 1
        l = np.zeros(len(a), np.float64)
        fail = self.lib.orc_ic0(n, rp, _ptr(ci), _ptr(a), _ptr(l))
        return l, int(fail)

    def ilu0(self, rp, ci, a):
        """Zero fill-in incomplete LU of A (Table 2, combination 6).

        Returns (L and U values in A's pattern -- L strictly below the
        diagonal with its unit diagonal implied, U on and above it --, first
        row with a zero or NaN pivot or -1)."""
        rp, ci, a = _i32(rp), _i32(ci), _f64(a)
        n = len(rp) - 1
        lu = np.zeros(len(a), np.float64)
        fail = self.lib.orc_ilu0(n, rp, _ptr(ci), _ptr(a), _ptr(lu))
        return lu, int(fail)

    def trsv_unit_lower(self, rp, ci, v, b):
        """y = L^{-1} b for the unit-lower L held in the strictly lower part."""
        rp, ci, v, b = _i32(rp), _i32(ci), _f64(v), _f64(b)
        n = len(rp) - 1
        y = np.zeros(n, np.float64)
        self.lib.orc_trsv_unit_lower(n, rp, _ptr(ci), _ptr(v), _ptr(b), _ptr(y))
        return y

    def backward(self, lrp, lci, lv, arp, aci, av, x, g):
        """Adjoint of y = A L^{-1} b: returns (grad_b, grad_L values)."""
        lrp, lci, lv = _i32(lrp), _i32(lci), _f64(lv)
        arp, aci, av = _i32(arp), _i32(aci), _f64(av)
        x, g = _f64(x), _f64(g)
        n = len(lrp) - 1
        m = len(arp) - 1
        gb = np.empty(n, np.float64)
        gl = np.empty(len(lv), np.float64)
        self.lib.orc_backward(n, m, lrp, _ptr(lci), _ptr(lv), arp, _ptr(aci), _ptr(av), _ptr(x),
                             _ptr(g), _ptr(gb), _ptr(gl))
        return gb, gl

    def levels(self, rp, ci):
        """Wavefront number of every SpTRSV row; returns (level, depth)."""
        rp, ci = _i32(rp), _i32(ci)
        n = len(rp) - 1
        lv = np.empty(n, np.int32)
        depth = self.lib.orc_levels(n, rp, _ptr(ci), _ptr(lv))
        return lv, int(depth)

    def reverse_levels(self, rp, ci):
        """Wavefront numbers of the transposed (upper) solve; returns (rlevel, depth)."""
        rp, ci = _i32(rp), _i32(ci)
        n = len(rp) - 1
        lv = np.empty(n, np.int32)
        depth = self.lib.orc_reverse_levels(n, rp, _ptr(ci), _ptr(lv))
        return lv, int(depth)

    def spmv_ready(self, arp, aci, level):
        """Joint level of every SpMV row with F = pattern(A)."""
        arp, aci, level = _i32(arp), _i32(aci), _i32(level)
        m = len(arp) - 1
        r = np.empty(m, np.int32)
        self.lib.orc_spmv_ready(m, arp, _ptr(aci), _ptr(level), _ptr(r))
        return r

    def joint_order_ts(self, level, ready):
        """Canonical joint order: (joint level, SpTRSV before SpMV, row)."""
        level, ready = _i32(level), _i32(ready)
        n, m = len(level), len(ready)
        order = np.empty(n + m, np.int32)
        self.lib.orc_joint_order_ts(n, _ptr(level), m, _ptr(ready), _ptr(order))
        return order

    def validate_ts(self, lrp, lci, arp, aci, order, item_ptr, allow_intra=False) -> int:
        """0 if the (order, item_ptr) schedule respects every edge, else a rule code."""
        lrp, lci, arp, aci = _i32(lrp), _i32(lci), _i32(arp), _i32(aci)
        order, item_ptr = _i32(order), _i32(item_ptr)
        return self.lib.orc_validate_ts(len(lrp) - 1, lrp, _ptr(lci), len(arp) - 1, arp, _ptr(aci),
                                       _ptr(order), len(item_ptr) - 1, item_ptr, int(allow_intra))

    def validate_factor_solve(self, rp, ci, order, item_ptr) -> int:
        """0 if the (order, item_ptr) schedule of a factorisation -> SpTRSV
        pair (ids 0..n-1 factor rows, n..2n-1 solve rows; F = I) respects
        every edge of the stored entries below the diagonal, else a rule
        code."""
        rp, ci, order, item_ptr = _i32(rp), _i32(ci), _i32(order), _i32(item_ptr)
        return self.lib.orc_validate_factor_solve(len(rp) - 1, rp, _ptr(ci), _ptr(order), len(item_ptr) - 1,
                                                  item_ptr)

    def validate_static_ts(self, lrp, lci, arp, aci, s_ptr, w_ptr, order) -> int:
        """0 if the two-level static schedule (s-partitions in sequence,
        independent w-partitions, each in its listed order) respects every
        edge of the joint SpTRSV -> SpMV DAG, else a rule code."""
        lrp, lci, arp, aci = _i32(lrp), _i32(lci), _i32(arp), _i32(aci)
        s_ptr, w_ptr, order = _i32(s_ptr), _i32(w_ptr), _i32(order)
        return self.lib.orc_validate_static_ts(len(lrp) - 1, lrp, _ptr(lci), len(arp) - 1, arp, _ptr(aci),
                                               len(s_ptr) - 1, s_ptr, len(w_ptr) - 1, w_ptr, _ptr(order))

    def reuse_ts(self, n, nnz_l, m, nnz_a) -> float:
        return float(self.lib.orc_reuse_ts(n, nnz_l, m, nnz_a))

    def reuse_it(self, n, nnz_l) -> float:
        return float(self.lib.orc_reuse_it(n, nnz_l))

    def refine(self, rp, ci, l64, arp, aci, a64, b, ncorr, l32=None):
        """Mixed-precision refinement of x = L^{-1} b (FP32 substitutions,
        FP64 residuals, ncorr corrections) and y = A x in FP64; see
        orc_refine.  l32 defaults to l64 rounded to FP32 (RNE).  Returns
        (x, y, relres, stages[n, ncorr + 1] as float32)."""
        rp, ci, l64, b = _i32(rp), _i32(ci), _f64(l64), _f64(b)
        arp, aci, a64 = _i32(arp), _i32(aci), _f64(a64)
        l32 = np.ascontiguousarray(l64.astype(np.float32) if l32 is None else l32, dtype=np.float32)
        n, m = len(rp) - 1, len(arp) - 1
        x = np.empty(max(n, 1), np.float64)
        y = np.empty(max(m, 1), np.float64)
        stages = np.empty((max(n, 1), ncorr + 1), np.float32)
        rel = self.lib.orc_refine(n, rp, _ptr(ci), _ptr(l64), _ptr(l32), m, arp, _ptr(aci), _ptr(a64),
                                  _ptr(b), int(ncorr), x, y, stages.ctypes.data)
        return x[:n], y[:m], float(rel), stages[:n]


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def __getattr__(name):
    # module-level access to the default oracle's routines: oracle.trsv_lower(...)
    if name.startswith("_"):
        raise AttributeError(name)
    return getattr(default(), name)
