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
