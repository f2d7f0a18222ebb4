"""The region plan of the fused SpTRSV -> SpMV executor (coarsen = 3): one
wavefront per region of up to a few hundred rows, x kept in LDS, every row
waiting only for its own inputs.  Results must be bit-identical to the
oracle (the arithmetic is forward substitution's, term by term)."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, dev_colmajor, host

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "lap3d7_24":
        A = synth.laplacian_3d7(24, 24, 24, 6.0)
    elif name == "lap2d9_64":
        A = synth.laplacian_2d9(64, 64, 8.0)
    elif name == "lap3d27_12":
        A = synth.laplacian_3d27(12, 12, 12, 26.1)
    elif name == "random":
        A = synth.random_spd(20_000, seed=8)
    elif name == "tridiag":
        A = synth.laplacian_1d(3000, 2.0)
    else:  # rectangular A with empty rows over a random lower L
        rng = np.random.default_rng(4)
        n = 4000
        Ld = sp.random(n, n, density=0.002, random_state=rng, format="csr")
        Ld.data[:] = rng.uniform(-1, 0, Ld.nnz)
        Ld = sp.tril(Ld, -1).tocsr() + sp.diags(rng.uniform(2, 3, n))
        Ad = sp.random(n + 9, n, density=0.002, random_state=rng, format="csr")
        Ad[::7] = 0
        Ad.eliminate_zeros()
        return synth.from_scipy(Ld.tocsr()), synth.from_scipy(Ad.tocsr())
    return synth.lower(A), A


def _oracle(orc, L, A, b):
    x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    return x, orc.spmv(A.rowptr, A.col, A.val, x)


@pytest.mark.parametrize("name,rows", [("lap3d7_24", 512), ("lap3d7_24", 64), ("lap2d9_64", 512),
                                       ("lap3d27_12", 512), ("random", 512), ("tridiag", 512), ("rect", 256)])
def test_region_plan_bit_identical(orc, name, rows):
    import torch
    L, A = _case(name)
    b = synth.vec_uniform(L.nrows, seed=1)
    s = sfm.Schedule(L, A, coarsen=3)
    if rows != 512:
        s.set_param("region_rows", rows)
    assert s.get_param("regioned") == 1
    announce("region plan %s rows=%d" % (name, rows))
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    xr, yr = _oracle(orc, L, A, b)
    assert np.array_equal(host(X), xr), name
    assert np.array_equal(host(Y), yr), name
    # SpTRSV alone (the region items only), and repeated launches
    announce("region plan %s: trsv only, repeated" % name)
    for _ in range(3):
        X2, _ = sfm.trsv_spmv(s, dev(L.val), None, dev(b), want_y=False)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    assert np.array_equal(host(X2), xr), name


@pytest.mark.parametrize("poll", [1, 7, 64 | (1 << 16), 64 | (64 << 16), 16 | (3 << 8) | (4 << 16), 64 | (2 << 16)])
@pytest.mark.parametrize("delay", [-1, 0, 3])
def test_region_poller_settings_bit_identical(orc, poll, delay):
    """The poller's lanes, first-input gate and back-off, and the SpMV rows'
    placement, change only when values are seen, never the results."""
    import torch
    L, A = _case("lap3d7_24")
    b = synth.vec_uniform(L.nrows, seed=3)
    s = sfm.Schedule(L, A, coarsen=3)
    s.set_param("region_poll", poll)
    s.set_param("spmv_delay", delay)
    assert s.get_param("region_poll") == poll and s.get_param("regioned") == 1
    announce("region poller %#x spmv_delay %d" % (poll, delay))
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    xr, yr = _oracle(orc, L, A, b)
    assert np.array_equal(host(X), xr)
    assert np.array_equal(host(Y), yr)


def test_region_plan_fp32_equals_level_plan():
    """FP32: the same per-row arithmetic as the level plan, so equal bits."""
    import torch
    L, A = _case("lap3d7_24")
    b = synth.vec_uniform(L.nrows, seed=2)
    s3 = sfm.Schedule(L, A, coarsen=3)
    s1 = sfm.Schedule(L, A, coarsen=1)
    Lv, Av, B = dev(L.val, torch.float32), dev(A.val, torch.float32), dev(b, torch.float32)
    announce("region plan fp32 vs level plan")
    X3, Y3 = sfm.trsv_spmv(s3, Lv, Av, B)
    X1, Y1 = sfm.trsv_spmv(s1, Lv, Av, B)
    torch.cuda.synchronize()
    sfm.sync_status(s3)
    sfm.sync_status(s1)
    assert np.array_equal(host(X3), host(X1)) and np.array_equal(host(Y3), host(Y1))


def test_region_plan_column_chains(orc):
    """Several right-hand sides as one chain of the region items per column."""
    import torch
    L, A = _case("lap2d9_64")
    b = synth.vec_uniform(L.nrows, k=3, seed=5)
    s = sfm.Schedule(L, A, coarsen=3)
    s.set_param("multi_path", 2)
    announce("region plan, 3 right-hand sides as column chains")
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev_colmajor(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    for c in range(3):
        xr, yr = _oracle(orc, L, A, b[:, c])
        assert np.array_equal(host(X)[:, c], xr) and np.array_equal(host(Y)[:, c], yr), c


def test_region_plan_trace_validity(orc):
    """Trace mode on the region plan: every region and SpMV item ran once,
    every row was published once, and each value reached every reader
    after its publication (inside a region: before the reader's own)."""
    import torch
    L, A = _case("lap3d7_24")
    n, m = L.nrows, A.nrows
    b = synth.vec_uniform(n, seed=1)
    s = sfm.Schedule(L, A, coarsen=3)
    s.set_param("trace", 1)
    announce("region plan trace")
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    xr, yr = _oracle(orc, L, A, b)
    assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr)
    items, rows = s.trace()
    level, order, ip = s.export()
    assert (items[:, 4] == 1).all() and (rows[:, 1] == 1).all()
    ready = items[:, 2].astype(np.int64)
    pub = rows[:, 0].astype(np.int64)
    item_of = np.repeat(np.arange(len(ip) - 1), np.diff(ip))[np.argsort(order, kind="stable")]
    ri = np.repeat(np.arange(n), np.diff(L.rowptr))
    off = L.col != ri
    i, j = ri[off], L.col[off]
    same = item_of[i] == item_of[j]
    assert same.any() and (~same).any()
    assert (ready[item_of[i[~same]]] >= pub[j[~same]]).all()
    assert (pub[j[same]] <= pub[i[same]]).all()
    rr = np.repeat(np.arange(m), np.diff(A.rowptr))
    assert (ready[item_of[n + rr]] >= pub[A.col]).all()


@pytest.mark.slow
def test_region_plan_full_size_128(orc):
    import torch
    L, A = synth.workload("lap3d7_128")
    b = synth.vec_uniform(L.nrows, seed=1)
    s = sfm.Schedule(L, A, coarsen=3)
    assert s.get_param("regioned") == 1
    announce("region plan lap3d7_128 full size")
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    xr, yr = _oracle(orc, L, A, b)
    assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr)
