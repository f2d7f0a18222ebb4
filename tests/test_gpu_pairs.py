"""GPU parity of the fused kernel combinations 1 (SpTRSV -> SpTRSV with one
L) and 2 (SpMV -> SpTRSV) of the paper's Table 2, and of the preconditioner
apply z = L^{-T} L^{-1} r, against the oracle's sequential kernels, on level,
coarsened and region plans: FP64 results bit for bit."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host, relerr

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "lap3d7_20":
        A = synth.laplacian_3d7(20, 20, 20, 6.0)
    elif name == "lap2d9_64":
        A = synth.laplacian_2d9(64, 64, 8.0)
    elif name == "random_spd":
        A = synth.random_spd(20000, seed=7)
    elif name == "ragged":
        n = 3001
        L = synth.random_lower(n, 0.003, seed=5)
        A = synth.from_scipy(sp.random(n, n, density=0.004, random_state=np.random.default_rng(6), format="csr"))
        return L, A
    else:
        return synth.workload(name)
    return synth.lower(A), A


CASES = ["lap2d5_64", "lap3d7_20", "lap2d9_64", "random_spd", "ragged"]


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("coarsen", [1, 2, 3])
def test_spmv_trsv_bit_identical(orc, name, coarsen):
    announce("pair spmv->trsv %s coarsen=%d" % (name, coarsen))
    import torch
    L, A = _case(name)
    x = synth.vec_uniform(L.nrows, seed=4)
    yr = orc.spmv(A.rowptr, A.col, A.val, x)
    zr = orc.trsv_lower(L.rowptr, L.col, L.val, yr)
    s = sfm.Schedule(L, A, coarsen=coarsen, rows_per_item=41)
    for unfused in (False, True):
        Y, Z = sfm.spmv_trsv(s, dev(A.val), dev(L.val), dev(x), unfused=unfused)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(Y), yr) and np.array_equal(host(Z), zr), unfused
    _, Z = sfm.spmv_trsv(s, dev(A.val), dev(L.val), dev(x), want_y=False)
    torch.cuda.synchronize()
    assert np.array_equal(host(Z), zr)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("coarsen", [1, 2, 3])
def test_trsv_trsv_bit_identical(orc, name, coarsen):
    announce("pair trsv->trsv %s coarsen=%d" % (name, coarsen))
    import torch
    L, A = _case(name)
    b = synth.vec_uniform(L.nrows, seed=8)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    zr = orc.trsv_lower(L.rowptr, L.col, L.val, xr)
    s = sfm.Schedule(L, A, coarsen=coarsen)
    for unfused in (False, True):
        X, Z = sfm.trsv_trsv(s, dev(L.val), dev(b), unfused=unfused)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(X), xr) and np.array_equal(host(Z), zr), unfused


def test_pairs_fp32_and_integer(orc):
    """FP32: within the forward-error bound of two solves; an integer
    manufactured case is exact in FP64 (every partial sum an integer)."""
    announce("pairs fp32 + integer")
    import torch
    A = synth.laplacian_3d7(16, 16, 16, 6.0)
    L = synth.lower(A)
    Li = synth.from_scipy(sp.csr_matrix((np.where(L.col == np.repeat(np.arange(L.nrows), np.diff(L.rowptr)),
                                                  1.0, -1.0), L.col, L.rowptr), shape=(L.nrows, L.nrows)))
    zt = synth.int_vector(L.nrows, seed=3)
    xt = Li.to_scipy() @ zt                     # L z = x  =>  z = L^{-1} x exactly
    bt = Li.to_scipy() @ xt
    s = sfm.Schedule(Li, A)
    X, Z = sfm.trsv_trsv(s, dev(Li.val), dev(bt))
    torch.cuda.synchronize()
    assert np.array_equal(host(X), xt) and np.array_equal(host(Z), zt)
    x = synth.vec_uniform(L.nrows, seed=4)
    yr = orc.spmv(A.rowptr, A.col, A.val, x)
    zr = orc.trsv_lower(L.rowptr, L.col, L.val, yr)
    s = sfm.Schedule(L, A)
    Y, Z = sfm.spmv_trsv(s, dev(A.val, torch.float32), dev(L.val, torch.float32), dev(x, torch.float32))
    torch.cuda.synchronize()
    # y: 7 terms rounded in FP32 (plus the FP32 rounding of inputs); z: a
    # diagonally dominant solve adds a modest factor
    assert relerr(host(Y), yr) < 1e-5 and relerr(host(Z), zr) < 1e-5


@pytest.mark.parametrize("name", ["lap3d7_128", "randspd_1m"])
def test_pairs_full_size(orc, name):
    announce("pairs full size " + name)
    import torch
    L, A = synth.workload(name)
    s = sfm.Schedule(L, A)
    x = synth.vec_uniform(L.nrows, seed=1)
    yr = orc.spmv(A.rowptr, A.col, A.val, x)
    zr = orc.trsv_lower(L.rowptr, L.col, L.val, yr)
    Y, Z = sfm.spmv_trsv(s, dev(A.val), dev(L.val), dev(x))
    torch.cuda.synchronize()
    assert np.array_equal(host(Y), yr) and np.array_equal(host(Z), zr)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, x)
    z2 = orc.trsv_lower(L.rowptr, L.col, L.val, xr)
    X, Z = sfm.trsv_trsv(s, dev(L.val), dev(x))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    assert np.array_equal(host(X), xr) and np.array_equal(host(Z), z2)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("coarsen", [1, 2, 3])
def test_ic_apply_bit_identical(orc, name, coarsen):
    """w = L^{-1} r, z = L^{-T} w with the factor's own IC0 values where the
    pattern admits one (else L's values): forward and backward substitution
    row by row, bit for bit, fused and unfused; with coarsen = 3 the fused
    apply on both region plans and on items."""
    announce("ic apply %s coarsen=%d" % (name, coarsen))
    import torch
    L, A = _case(name)
    lv, fail = orc.ic0(L.rowptr, L.col, L.val)
    if fail >= 0:
        lv = L.val
    r = synth.vec_normal(L.nrows, seed=9)
    wr = orc.trsv_lower(L.rowptr, L.col, lv, r)
    zr = orc.trsv_upper_t(L.rowptr, L.col, lv, wr)
    s = sfm.Schedule(L, A, coarsen=coarsen, want_backward=True)
    if coarsen == 3:
        assert s.get_param("regioned") == 1 and s.get_param("back_regioned") == 1
    for pr in ((1, 0) if coarsen == 3 else (1,)):
        s.set_param("precond_regions", pr)
        for unfused in (False, True):
            W, Z = sfm.ic_apply(s, dev(lv), dev(r), unfused=unfused)
            torch.cuda.synchronize()
            sfm.sync_status(s)
            assert np.array_equal(host(W), wr) and np.array_equal(host(Z), zr), (pr, unfused)


def test_ic_apply_fp32_regions_equal_items():
    """FP32: the apply on the region plans does each row's arithmetic in the
    same order as on items, so equal bits; both within FP32 rounding of the
    FP64 result."""
    announce("ic apply fp32 regions vs items lap3d7_20")
    import torch
    L, A = _case("lap3d7_20")
    r = synth.vec_normal(L.nrows, seed=5)
    s = sfm.Schedule(L, A, coarsen=3, want_backward=True)
    assert s.get_param("regioned") == 1 and s.get_param("back_regioned") == 1
    out = {}
    for pr in (1, 0):
        s.set_param("precond_regions", pr)
        W, Z = sfm.ic_apply(s, dev(L.val, torch.float32), dev(r, torch.float32))
        torch.cuda.synchronize()
        sfm.sync_status(s)
        out[pr] = (host(W), host(Z))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    s.set_param("precond_regions", 1)
    W64, Z64 = sfm.ic_apply(s, dev(L.val), dev(r))
    torch.cuda.synchronize()
    z64 = host(Z64)
    assert np.max(np.abs(out[1][1] - z64)) <= 1e-4 * np.max(np.abs(z64))


def test_ic_apply_full_size(orc):
    announce("ic apply full size lap3d7_96")
    import torch
    L, A = synth.workload("lap3d7_96")
    lv, fail = orc.ic0(L.rowptr, L.col, L.val)
    assert fail == -1
    r = synth.vec_normal(L.nrows, seed=9)
    wr = orc.trsv_lower(L.rowptr, L.col, lv, r)
    zr = orc.trsv_upper_t(L.rowptr, L.col, lv, wr)
    s = sfm.Schedule(L, A, want_backward=True)
    assert s.get_param("regioned") == 1 and s.get_param("back_regioned") == 1  # the region apply
    for rep in range(2):
        W, Z = sfm.ic_apply(s, dev(lv), dev(r))
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(W), wr) and np.array_equal(host(Z), zr), rep
