"""FP32 fused solves with FP64 residual refinement: after the corrections,
x and y = A x agree with the FP64 oracle to 1e-10 normwise relative per
right-hand side; the pure FP32 pass alone does not."""
import numpy as np
import pytest

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, dev_colmajor, host, relerr

pytestmark = pytest.mark.gpu
TOL_REFINED = 1e-10


def run_refine(s, L, A, b, n_corr):
    import torch
    L64, A64 = dev(L.val), dev(A.val)
    L32 = dev(L.val, torch.float32)
    B = dev(b) if b.ndim == 1 else dev_colmajor(b)
    X, Y, rel = sfm.refine_trsv_spmv(s, L32, L64, A64, B, n_corrections=n_corr)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    return host(X), host(Y), rel


def oracle_cols(orc, L, A, b):
    bb = b if b.ndim == 2 else b[:, None]
    xs = np.stack([orc.trsv_lower(L.rowptr, L.col, L.val, bb[:, c]) for c in range(bb.shape[1])], 1)
    ys = np.stack([orc.spmv(A.rowptr, A.col, A.val, xs[:, c]) for c in range(bb.shape[1])], 1)
    return (xs[:, 0], ys[:, 0]) if b.ndim == 1 else (xs, ys)


@pytest.mark.parametrize("mat,k", [("spd", 1), ("spd", 8), ("spd", 13), ("9pt", 1), ("9pt", 32)])
def test_refinement_reaches_1e10(orc, mat, k):
    announce("refine %s k=%d" % (mat, k))
    if mat == "spd":
        A = synth.random_spd(100_000, seed=0)
    else:
        A = synth.laplacian_2d9(256, 256, 8.0)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, k=k, seed=1)
    s = sfm.Schedule(L, A)
    xr, yr = oracle_cols(orc, L, A, b)
    x0, y0, _ = run_refine(s, L, A, b, 0)
    x, y, rel = run_refine(s, L, A, b, 2)
    print("%s k=%d: fp32-only x err %.2e; refined x err %.2e y err %.2e relres %.2e"
          % (mat, k, relerr(x0, xr), relerr(x, xr), relerr(y, yr), rel.max()))
    assert relerr(x0, xr) > 1e-9          # one FP32 pass is not accurate enough
    assert relerr(x, xr) <= TOL_REFINED
    assert relerr(y, yr) <= TOL_REFINED
    assert rel.max() <= 1e-12


# ---- the batched workloads at full size: random SPD n = 10^6 and the 2D
# 9-point Laplacian on a 2048^2 grid, k in {1, 8, 32, 64} right-hand sides
# (b ~ U(-1, 1), seed 1), every column compared with the FP64 oracle

_FULL = {}


def full_case(orc, mat):
    """(L, A, b[:, :64], x_oracle, y_oracle) for a full-size batched
    workload, computed once per session (64 sequential oracle solves)."""
    if mat not in _FULL:
        L, A = synth.workload("randspd_1m" if mat == "spd" else "lap2d9_2048")
        b = synth.vec_uniform(L.nrows, k=64, seed=1)
        xr, yr = oracle_cols(orc, L, A, b)
        _FULL.clear()  # keep one matrix's arrays at a time
        _FULL[mat] = (L, A, b, xr, yr)
    return _FULL[mat]


@pytest.mark.slow
@pytest.mark.parametrize("mat", ["spd", "9pt"])
def test_full_size_refinement_every_k(orc, mat):
    """FP32 solves (block widths up to 64) + 2 FP64 corrections reach 1e-10
    against the FP64 oracle in x and y, per column, at k = 1, 8, 32, 64 on
    the full-size batched matrices; relative residuals <= 1e-12."""
    L, A, b, xr, yr = full_case(orc, mat)
    s = sfm.Schedule(L, A)
    for k in (1, 8, 32, 64):
        announce("refine full-size %s k=%d" % (mat, k))
        bk = b[:, 0] if k == 1 else b[:, :k]
        x, y, rel = run_refine(s, L, A, bk, 2)
        xk = xr[:, 0] if k == 1 else xr[:, :k]
        yk = yr[:, 0] if k == 1 else yr[:, :k]
        ex, ey = relerr(x, xk), relerr(y, yk)
        print("%s k=%d refined: x err %.2e  y err %.2e  relres %.2e" % (mat, k, ex, ey, rel.max()))
        assert ex <= TOL_REFINED and ey <= TOL_REFINED, (k, ex, ey)
        assert rel.max() <= 1e-12, (k, rel.max())
    s.free()


@pytest.mark.slow
@pytest.mark.parametrize("mat", ["spd", "9pt"])
def test_full_size_fp64_k64_bit_identical(orc, mat):
    """FP64 fused SpTRSV -> SpMV with 64 right-hand sides in one launch
    (interleaved blocks of 64 columns) and the unfused level-set baseline:
    every column of x and y bit-identical to the oracle, full size."""
    import torch
    L, A, b, xr, yr = full_case(orc, mat)
    s = sfm.Schedule(L, A)
    Lv, Av, B = dev(L.val), dev(A.val), dev_colmajor(b)
    for unfused in (False, True):
        announce("fp64 k=64 full-size %s unfused=%s" % (mat, unfused))
        X, Y = sfm.trsv_spmv(s, Lv, Av, B, unfused=unfused)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(X), xr), unfused
        assert np.array_equal(host(Y), yr), unfused
        del X, Y
    s.free()


def test_fp32_kb64_refinement_small(orc):
    """The 64-wide FP32 kernels (solve units, pack with conversion,
    residual and final passes on 64-column blocks) on a small random SPD
    matrix: refined x and y within 1e-10 of the oracle, per column."""
    A = synth.random_spd(20_000, seed=4)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, k=64, seed=1)
    s = sfm.Schedule(L, A)
    assert s.get_param("rhs_block") == 0  # default block width for 64 columns is 64
    xr, yr = oracle_cols(orc, L, A, b)
    for nc in (1, 2, 3):
        announce("refine fp32 kb=64 n=20000 corrections=%d" % nc)
        x, y, rel = run_refine(s, L, A, b, nc)
        assert relerr(x, xr) <= TOL_REFINED and relerr(y, yr) <= TOL_REFINED, nc
        assert rel.max() <= 1e-12, nc


# ---- the fused refinement (one launch: FP32 substitution, corrections,
# final residual and y = A x) against the refinement oracle, bit for bit

def oracle_refine_cols(orc, L, A, b, nc):
    bb = b if b.ndim == 2 else b[:, None]
    outs = [orc.refine(L.rowptr, L.col, L.val, A.rowptr, A.col, A.val, bb[:, c], nc) for c in range(bb.shape[1])]
    xs = np.stack([o[0] for o in outs], 1)
    ys = np.stack([o[1] for o in outs], 1)
    rel = np.array([o[2] for o in outs])
    if b.ndim == 1:
        return xs[:, 0], ys[:, 0], rel
    return xs, ys, rel


@pytest.mark.parametrize("mat,k,nc", [("spd", 1, 0), ("spd", 1, 1), ("spd", 1, 2), ("spd", 1, 3),
                                      ("9pt", 1, 2), ("spd", 5, 2), ("spd", 8, 1), ("9pt", 32, 2),
                                      ("spd", 64, 3), ("ragged", 3, 2), ("ragged", 1, 1)])
def test_fused_refinement_bit_identical_to_oracle(orc, mat, k, nc):
    if mat == "spd":
        A = synth.random_spd(20_000, seed=3)
    elif mat == "9pt":
        A = synth.laplacian_2d9(96, 80, 8.0)
    else:  # rows of very different lengths, empty SpMV rows, rectangular A
        import scipy.sparse as sp
        rng = np.random.default_rng(9)
        n = 3000
        Ld = sp.random(n, n, density=0.004, random_state=rng, format="csr")
        Ld.data[:] = rng.uniform(-1, 0, Ld.nnz)
        Ld = sp.tril(Ld, -1).tocsr()
        Ld[np.arange(0, n, 97), :60] = -0.01  # a few long rows
        Ld = sp.tril(Ld, -1).tocsr()
        Ld = Ld + sp.diags(1.0 + abs(Ld).sum(1).A1)
        Ad = sp.random(n + 7, n, density=0.003, random_state=rng, format="csr")
        Ad[::11] = 0
        Ad.eliminate_zeros()
        L, A0 = synth.from_scipy(Ld.tocsr()), synth.from_scipy(Ad.tocsr())
        A = None
    if A is not None:
        L = synth.lower(A)
        A0 = A
    b = synth.vec_uniform(L.nrows, k=k, seed=1)
    s = sfm.Schedule(L, A0, coarsen=1)  # level items: the fused refinement's plan
    announce("fused refine %s k=%d nc=%d" % (mat, k, nc))
    x, y, rel = run_refine(s, L, A0, b, nc)
    xr, yr, relr = oracle_refine_cols(orc, L, A0, b, nc)
    assert np.array_equal(x, xr), (mat, k, nc, relerr(x, xr))
    assert np.array_equal(y, yr), (mat, k, nc, relerr(y, yr))
    assert np.array_equal(rel, relr), (rel, relr)


def test_staged_refinement_path_still_reaches_1e10(orc):
    """The staged refinement (one launch per pass) stays available as the
    comparison path (refine_path = 1)."""
    A = synth.random_spd(30_000, seed=0)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, k=8, seed=1)
    s = sfm.Schedule(L, A)
    s.set_param("refine_path", 1)
    xr, yr = oracle_cols(orc, L, A, b)
    announce("staged refine spd k=8")
    x, y, rel = run_refine(s, L, A, b, 2)
    assert relerr(x, xr) <= TOL_REFINED and relerr(y, yr) <= TOL_REFINED and rel.max() <= 1e-12
