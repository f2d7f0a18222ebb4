"""Argument checks of the Python binding, made before any library call: every
value array and vector must share the executor's dtype and device, value
arrays must hold exactly the stored entries of the inspected pattern and be
contiguous, vectors must have unit stride down each column.  The checks run
on CPU tensors here (the last check, that the tensors sit on a GPU, is what a
fully consistent CPU call reports), so no device buffer is ever handed to the
library with a wrong size."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2111_12238_amd as sfm
import synth


@pytest.fixture(scope="module")
def ts():
    L, A = synth.workload("lap2d5_16")
    return sfm.Schedule(L, A, want_backward=True), L, A


def cpu(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt)


def raises(fn, match):
    with pytest.raises(ValueError, match=match):
        fn()


def test_trsv_spmv_mismatches(ts):
    s, L, A = ts
    n = L.nrows
    Lv, Av, b = cpu(L.val), cpu(A.val), cpu(np.ones(n))
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, b), "GPU device")  # consistent, but on the host
    raises(lambda: sfm.trsv_spmv(s, Lv, cpu(A.val, torch.float32), b), "A_val: dtype")
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, cpu(np.ones(n), torch.float32)), "B: dtype")
    raises(lambda: sfm.trsv_spmv(s, Lv[:-1], Av, b), "L_val has %d values" % (L.nnz - 1))
    raises(lambda: sfm.trsv_spmv(s, Lv, torch.cat([Av, Av[:1]]), b), "A_val has")
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, b, X=torch.empty(n, dtype=torch.float32)), "X: dtype")
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, b, Y=torch.empty(n + 1, dtype=torch.float64)), "Y: expected")
    strided = torch.empty(2 * L.nnz, dtype=torch.float64)[::2]
    raises(lambda: sfm.trsv_spmv(s, strided, Av, b), "L_val must be contiguous")
    with pytest.raises(TypeError):
        sfm.trsv_spmv(s, Lv.to(torch.int64), Av, b)


def test_strided_column_views_rejected(ts):
    """A (n, 1) column of a row-major (n, 2) tensor has stride (2, 1): it
    must be refused (not read as if contiguous), as input and as output."""
    s, L, A = ts
    n = L.nrows
    Lv, Av = cpu(L.val), cpu(A.val)
    two = torch.zeros(n, 2, dtype=torch.float64)
    col = two[:, 1:2]
    assert col.stride() == (2, 1)
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, col), "B: rows must be contiguous")
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, cpu(np.ones(n)), X=col), "X: expected a contiguous vector|X: rows")
    B2 = torch.zeros(2, n, dtype=torch.float64).t()  # proper column-major (n, 2)
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, B2, X=torch.zeros(2, n, dtype=torch.float64).t(),
                                 Y=torch.zeros(3, n, dtype=torch.float64).t()), "same number of columns")
    raises(lambda: sfm.trsv_spmv(s, Lv, Av, torch.zeros(n, 2, dtype=torch.float64)),
           "rows must be contiguous")


def test_other_executors_mismatches(ts):
    s, L, A = ts
    n = L.nrows
    Lv, Av, b = cpu(L.val), cpu(A.val), cpu(np.ones(n))
    f32 = cpu(np.ones(n), torch.float32)
    raises(lambda: sfm.spmv_trsv(s, Av, Lv, f32), "x: dtype")
    raises(lambda: sfm.trsv_trsv(s, Lv, f32), "b: dtype")
    raises(lambda: sfm.ic_apply(s, Lv[:3], b), "L_val has 3 values")
    raises(lambda: sfm.static_trsv_spmv(s, sfm.SF_STATIC_MSP, Lv, Av[:5], b), "A_val has 5")
    raises(lambda: sfm.backward(s, Lv, Av, f32, X=b), "G: dtype")
    raises(lambda: sfm.backward(s, Lv, Av, b), "needs X")
    raises(lambda: sfm.backward(s, Lv, Av, b, X=b), "GPU device")
    raises(lambda: sfm.refine_trsv_spmv(s, Lv, Lv, Av, b), "L32: dtype")
    raises(lambda: sfm.refine_trsv_spmv(s, Lv.float(), Lv.float(), Av, b), "L64: dtype")
    raises(lambda: sfm.refine_trsv_spmv(s, Lv.float(), Lv, Av, f32), "B: dtype")
    raises(lambda: sfm.refine_trsv_spmv(s, Lv.float(), Lv, Av, b), "GPU device")
    raises(lambda: sfm.autotune(s, Lv, Av, f32), "B: dtype")


def test_factorisation_executors_mismatches():
    a = synth.laplacian_3d27(4, 4, 4, 26.1)
    Lp = synth.lower(a)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    v = cpu(Lp.val)
    raises(lambda: sfm.ic0_trsv(s, v.float()), "A_lower_val: dtype")
    raises(lambda: sfm.ic0_trsv(s, v[:-2]), "A_lower_val has")
    raises(lambda: sfm.ic0_trsv(s, v, cpu(np.ones(Lp.nrows), torch.float32)), "b: dtype")
    raises(lambda: sfm.ic0_trsv(s, v, L_val=torch.empty(3, dtype=torch.float64)), "L_val has 3")
    raises(lambda: sfm.ic0_trsv(s, v, cpu(np.ones(Lp.nrows))), "GPU device")
    c = synth.convdiff_3d7(4, 4, 4)
    si = sfm.Schedule(c, None, sfm.SF_ILU0_TRSV)
    raises(lambda: sfm.ilu0_trsv(si, cpu(c.val, torch.float32)), "A_val: dtype")
    raises(lambda: sfm.ilu0_trsv(si, cpu(c.val), cpu(np.ones(c.nrows + 1))), "x: expected")


def test_multi_rhs_offset_limit_is_host_side():
    """Several right-hand sides address a block's interleaved x with 32-bit
    offsets: n * rhs_block >= 2^31 (2^25 rows, 64 right-hand sides) is
    reported as SF_ERR_UNSUPPORTED by the fused and level-set entries from
    the schedule alone -- before the buffer pointers (NULL here) are looked
    at, so no device memory is involved."""
    n = 1 << 25
    rp = np.arange(n + 1, dtype=np.int32)
    s = sfm.Schedule((rp, rp[:-1].copy(), n), (np.zeros(1, np.int32), np.zeros(0, np.int32), n))
    assert s.info().coarsened == 0 and s.get_param("multi_path") == 0  # interleaved units for 64 RHS
    lib = sfm._lib()
    for fn in (lib.sf_exec_trsv_spmv, lib.sf_exec_unfused_trsv_spmv):
        assert fn(s.handle, 0, None, None, None, n, 64, None, n, None, 0, None) == 10  # SF_ERR_UNSUPPORTED
        # at 32 right-hand sides the offsets fit: the NULL buffers are then reported
        assert fn(s.handle, 0, None, None, None, n, 32, None, n, None, 0, None) == 1  # SF_ERR_ARG
    s.free()


def test_autotune_fingerprint_tells_patterns_apart():
    """The autotuner's cache key, host-side: equal patterns share a fingerprint, a changed column or a
    different size does not."""
    A = synth.laplacian_2d5(20, 20, 4.0)
    L = synth.lower(A)
    f1 = sfm.Schedule(L, A).get_param("fingerprint")
    f2 = sfm.Schedule(L, A).get_param("fingerprint")
    A3 = synth.laplacian_2d9(20, 20, 8.0)
    f3 = sfm.Schedule(synth.lower(A3), A3).get_param("fingerprint")
    assert f1 == f2 and f1 != f3


def test_noalloc_backward_size_limit_is_host_side():
    """The allocation-free adjoint keeps a recomputed x in a fixed 64 MiB
    device scratch: a system of more than 2^23 rows (FP64) is refused with
    SF_ERR_UNSUPPORTED from the schedule alone, before any pointer or device
    is looked at; FP32 fits twice as many rows."""
    P, I = ctypes.c_void_p, ctypes.c_int32
    lib = sfm._lib()
    f = lib.sf_backward_noalloc
    f.argtypes = [P, I, P, P, P, P, P, P, P, P]
    f.restype = ctypes.c_int
    n = (1 << 23) + 1
    rp = np.arange(n + 1, dtype=np.int32)
    s = sfm.Schedule((rp, rp[:-1].copy(), n), (rp, rp[:-1].copy(), n), want_backward=True)
    fake = ctypes.c_void_p(0x1000)
    assert f(s.handle, 0, fake, fake, None, fake, fake, fake, fake, None) == 10  # SF_ERR_UNSUPPORTED
    s.free()
