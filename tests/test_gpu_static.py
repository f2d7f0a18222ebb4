"""GPU parity of the static schedules (the paper's fused partitioning, MSP,
and the fused wavefront baseline) against the oracle's sequential kernels:
FP64 x and y bit for bit, FP32 equal to the dynamic executor's FP32 result
(same per-row arithmetic in every schedule)."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

PLANS = [sfm.SF_STATIC_MSP, sfm.SF_STATIC_WAVEFRONT]


def _case(name):
    if name == "random":
        L = synth.random_lower(3001, 0.003, seed=5)
        A = synth.from_scipy(sp.random(2000, 3001, density=0.002, random_state=np.random.default_rng(2),
                                       format="csr"))
        return L, A
    if name == "chains":
        blk = sp.diags([np.full(49, -1.0), np.full(50, 2.0)], [-1, 0])
        L = synth.from_scipy(sp.block_diag([blk] * 8, format="csr"))
        return L, synth.from_scipy(sp.random(400, 400, density=0.01, random_state=np.random.default_rng(4),
                                             format="csr"))
    if name == "random_spd":
        A = synth.random_spd(30000, seed=5)
        return synth.lower(A), A
    if name == "lap3d7_20":
        A = synth.laplacian_3d7(20, 20, 20, 6.0)
        return synth.lower(A), A
    return synth.workload(name)


@pytest.mark.parametrize("name", ["lap2d5_64", "random", "chains", "random_spd", "lap3d7_20"])
@pytest.mark.parametrize("plan", PLANS)
def test_static_bit_identical(orc, name, plan):
    announce("static plan %d %s" % (plan, name))
    import torch
    L, A = _case(name)
    b = synth.vec_uniform(L.nrows, seed=3)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    yr = orc.spmv(A.rowptr, A.col, A.val, xr)
    s = sfm.Schedule(L, A)
    for _ in range(2):  # a second launch reuses the plan and the state block
        X, Y = sfm.static_trsv_spmv(s, plan, dev(L.val), dev(A.val), dev(b))
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr)
    # FP32: the same arithmetic as the dynamic executor, so equal bit for bit
    L32, A32, b32 = (dev(v, torch.float32) for v in (L.val, A.val, b))
    X, Y = sfm.static_trsv_spmv(s, plan, L32, A32, b32)
    Xf, Yf = sfm.trsv_spmv(s, L32, A32, b32)
    torch.cuda.synchronize()
    assert torch.equal(X, Xf) and torch.equal(Y, Yf)


def test_static_msp_parts_and_full_size(orc):
    """A different number of w-partitions per s-partition rebuilds the MSP
    plan; the 3D 7-point 128^3 workload is exact under both plans."""
    announce("static plans msp_parts and 128^3")
    import torch
    L, A = synth.workload("lap2d5_64")
    b = synth.vec_uniform(L.nrows, seed=8)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    yr = orc.spmv(A.rowptr, A.col, A.val, xr)
    s = sfm.Schedule(L, A)
    for parts in (1, 7, 4096):
        s.set_param("msp_parts", parts)
        X, Y = sfm.static_trsv_spmv(s, sfm.SF_STATIC_MSP, dev(L.val), dev(A.val), dev(b))
        torch.cuda.synchronize()
        assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr), parts
    L, A = synth.workload("lap3d7_128")
    b = synth.vec_uniform(L.nrows, seed=1)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    yr = orc.spmv(A.rowptr, A.col, A.val, xr)
    s = sfm.Schedule(L, A)
    Lv, Av, B = dev(L.val), dev(A.val), dev(b)
    for plan in PLANS:
        X, Y = sfm.static_trsv_spmv(s, plan, Lv, Av, B)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr), plan


def test_static_degenerate(orc):
    """One row; a diagonal L (one wavefront, one s-partition); an A without
    rows (no Y): exact results under both plans."""
    announce("static plans degenerate")
    import torch
    cases = [
        (sp.csr_matrix(np.array([[2.0]])), sp.csr_matrix(np.array([[3.0]]))),
        (sp.identity(50, format="csr") * 2.0, sp.random(30, 50, density=0.1, random_state=np.random.default_rng(1),
                                                         format="csr")),
        (sp.identity(20, format="csr") + sp.eye(20, k=-1, format="csr"), sp.csr_matrix((0, 20))),
    ]
    for ld, ad in cases:
        L, A = synth.from_scipy(sp.csr_matrix(ld)), synth.from_scipy(sp.csr_matrix(ad))
        b = synth.vec_uniform(L.nrows, seed=2)
        xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
        s = sfm.Schedule(L, A)
        for plan in PLANS:
            Av = dev(A.val) if A.nnz else None
            X, Y = sfm.static_trsv_spmv(s, plan, dev(L.val), Av, dev(b))
            torch.cuda.synchronize()
            sfm.sync_status(s)
            assert np.array_equal(host(X), xr), plan
            if A.nrows:
                assert np.array_equal(host(Y), orc.spmv(A.rowptr, A.col, A.val, xr)), plan
            else:
                assert Y is None
