"""GPU parity of the adjoint executor: grad_b = L^{-T} A^T g and
grad_L = -(grad_b x^T) on the pattern of L, against the oracle (itself
pinned by finite differences and dense formulas), through the C ABI and
through torch.autograd."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host, relerr

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def oracle_grads(orc, L, A, b, w):
    x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    gb, gl = orc.backward(L.rowptr, L.col, L.val, A.rowptr, A.col, A.val, x, w)
    return x, gb, gl


def gpu_grads(s, L, A, b, w, dtype=None, recompute=False):
    import torch
    dtype = dtype or torch.float64
    Lv, Av, B, G = dev(L.val, dtype), dev(A.val, dtype), dev(b, dtype), dev(w, dtype)
    X, _ = sfm.trsv_spmv(s, Lv, Av, B, want_y=False)
    if recompute:
        gb, gl = sfm.backward(s, Lv, Av, G, B=B)
    else:
        gb, gl = sfm.backward(s, Lv, Av, G, X=X)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    return host(gb), host(gl)


def test_lap2d5_16(orc):
    announce("bwd lap2d5_16")
    L, A = synth.workload("lap2d5_16")
    b = synth.vec_uniform(L.nrows, seed=1)
    w = synth.vec_normal(A.nrows, seed=2)
    s = sfm.Schedule(L, A, want_backward=True)
    _, gbr, glr = oracle_grads(orc, L, A, b, w)
    gb, gl = gpu_grads(s, L, A, b, w)
    assert relerr(gb, gbr) <= TOL64 and relerr(gl, glr) <= TOL64
    # the adjoint runs the definition's terms in its order: equal bit for bit
    assert np.array_equal(gb, gbr) and np.array_equal(gl, glr)
    gb2, gl2 = gpu_grads(s, L, A, b, w, recompute=True)
    assert np.array_equal(gb, gb2) and np.array_equal(gl, gl2)


@pytest.mark.parametrize("seed,n,m,lanes", [(0, 3000, 2000, 4), (1, 777, 1500, 16), (2, 5000, 5000, 32)])
def test_random_rectangular(orc, seed, n, m, lanes):
    announce("bwd random n=%d m=%d lanes=%d" % (n, m, lanes))
    L = synth.random_lower(n, min(0.5, 5.0 / n), seed=seed)
    a = sp.random(m, n, density=min(1.0, 7.0 / n), random_state=np.random.default_rng(seed), format="csr")
    A = synth.from_scipy(a)
    b = synth.vec_uniform(n, seed=seed + 1)
    w = synth.vec_normal(m, seed=seed + 2)
    s = sfm.Schedule(L, A, want_backward=True, lanes_per_row=lanes, rows_per_item=29)
    _, gbr, glr = oracle_grads(orc, L, A, b, w)
    gb, gl = gpu_grads(s, L, A, b, w)
    assert relerr(gb, gbr) <= TOL64 and relerr(gl, glr) <= TOL64


@pytest.mark.parametrize("case", ["lap3d7_16", "lap2d9_48", "lap2d5_16"])
def test_coarsened_backward_bit_identical(orc, case):
    """Coarsened items in the transposed solve (lambda values of an item
    resolved in LDS) keep the definition's arithmetic: FP64 gradients equal
    the oracle's bit for bit, also with a small item size."""
    announce("bwd coarsened " + case)
    if case == "lap3d7_16":
        A = synth.laplacian_3d7(16, 16, 16, 6.0)
        L = synth.lower(A)
    elif case == "lap2d9_48":
        A = synth.laplacian_2d9(48, 48, 8.0)
        L = synth.lower(A)
    else:
        L, A = synth.workload("lap2d5_16")
    b = synth.vec_uniform(L.nrows, seed=1)
    w = synth.vec_normal(A.nrows, seed=2)
    _, gbr, glr = oracle_grads(orc, L, A, b, w)
    for rows in (64, 11):
        s = sfm.Schedule(L, A, want_backward=True, coarsen=2, rows_per_item=rows)
        assert s.info().back_coarsened == 1
        gb, gl = gpu_grads(s, L, A, b, w)
        assert np.array_equal(gb, gbr) and np.array_equal(gl, glr), rows
        gb2, gl2 = gpu_grads(s, L, A, b, w, recompute=True)
        assert np.array_equal(gb2, gbr) and np.array_equal(gl2, glr), rows


def test_autograd_function(orc):
    announce("bwd autograd lap2d5_16")
    import torch
    L, A = synth.workload("lap2d5_16")
    b = synth.vec_uniform(L.nrows, seed=1)
    w = synth.vec_normal(A.nrows, seed=2)
    s = sfm.Schedule(L, A, want_backward=True)
    _, gbr, glr = oracle_grads(orc, L, A, b, w)
    for recompute in (False, True):
        Lv = dev(L.val).requires_grad_(True)
        B = dev(b).requires_grad_(True)
        y = sfm.trsv_spmv_autograd(Lv, B, dev(A.val), s, recompute)
        loss = (y * dev(w)).sum()
        loss.backward()
        torch.cuda.synchronize()
        assert relerr(host(B.grad), gbr) <= TOL64
        assert relerr(host(Lv.grad), glr) <= TOL64
        x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
        assert abs(loss.item() - w @ orc.spmv(A.rowptr, A.col, A.val, x)) <= 1e-12 * abs(loss.item())


def test_s5_lap3d7_96(orc):
    """Forward + backward at the 96^3 workload size, FP64 and FP32."""
    announce("bwd full size lap3d7_96")
    import torch
    L, A = synth.workload("lap3d7_96")
    b = synth.vec_uniform(L.nrows, seed=1)
    w = synth.vec_normal(A.nrows, seed=2)
    s = sfm.Schedule(L, A, want_backward=True)
    print("96^3 plans: forward coarsened %d, backward coarsened %d" % (s.info().coarsened, s.info().back_coarsened))
    _, gbr, glr = oracle_grads(orc, L, A, b, w)
    gb, gl = gpu_grads(s, L, A, b, w)
    print("96^3 FP64 grad errors: b %.2e L %.2e" % (relerr(gb, gbr), relerr(gl, glr)))
    assert relerr(gb, gbr) <= TOL64 and relerr(gl, glr) <= TOL64
    assert np.array_equal(gb, gbr) and np.array_equal(gl, glr)
    gb32, gl32 = gpu_grads(s, L, A, b, w, dtype=torch.float32)
    print("96^3 FP32 grad errors vs FP64 oracle: b %.2e L %.2e" % (relerr(gb32, gbr), relerr(gl32, glr)))
    assert relerr(gb32, gbr) < 1e-4 and relerr(gl32, glr) < 1e-4


@pytest.mark.parametrize("case", ["lap3d7_16", "lap2d9_48", "lap3d27_10", "random"])
def test_region_backward_bit_identical(orc, case):
    """The backward region plan (regions of the transposed solve on a
    computing and a polling wavefront, c_i staged with the rows, grad_L
    written after each region): FP64 gradients equal the oracle's bit for
    bit, with large and small regions, x given or recomputed; FP32 within
    rounding of the FP64 oracle."""
    import torch
    announce("bwd regions " + case)
    if case == "lap3d7_16":
        A = synth.laplacian_3d7(16, 16, 16, 6.0)
        L = synth.lower(A)
    elif case == "lap2d9_48":
        A = synth.laplacian_2d9(48, 48, 8.0)
        L = synth.lower(A)
    elif case == "lap3d27_10":
        A = synth.laplacian_3d27(10, 10, 10, 26.1)
        L = synth.lower(A)
    else:
        L = synth.random_lower(3000, 5.0 / 3000, seed=4)
        A = synth.from_scipy(sp.random(2000, 3000, density=7.0 / 3000, random_state=np.random.default_rng(4),
                                       format="csr"))
    b = synth.vec_uniform(L.nrows, seed=1)
    w = synth.vec_normal(A.nrows, seed=2)
    _, gbr, glr = oracle_grads(orc, L, A, b, w)
    for rows in (512, 64):
        s = sfm.Schedule(L, A, want_backward=True, coarsen=3)
        s.set_param("region_rows", rows)
        assert s.get_param("back_regioned") == 1
        gb, gl = gpu_grads(s, L, A, b, w)
        assert np.array_equal(gb, gbr) and np.array_equal(gl, glr), rows
        gb2, gl2 = gpu_grads(s, L, A, b, w, recompute=True)
        assert np.array_equal(gb2, gbr) and np.array_equal(gl2, glr), rows
    gb32, gl32 = gpu_grads(s, L, A, b, w, dtype=torch.float32)
    assert relerr(gb32, gbr) < 1e-4 and relerr(gl32, glr) < 1e-4
