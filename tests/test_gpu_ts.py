"""GPU parity of the fused SpTRSV -> SpMV executor (and its unfused
baseline) against the oracle.  FP64 tolerance: 1e-12 normwise relative;
integer manufactured solutions must match bit for bit."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, dev_colmajor, host, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def run(s, L, A, b, dtype="f64", unfused=False, k=None):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    Lv, Av = dev(L.val, td), dev(A.val, td)
    B = dev(b, td) if b.ndim == 1 else dev_colmajor(b, td)
    X, Y = sfm.trsv_spmv(s, Lv, Av, B, unfused=unfused)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    return host(X), host(Y)


def oracle_ts(orc, L, A, b):
    if b.ndim == 1:
        x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
        return x, orc.spmv(A.rowptr, A.col, A.val, x)
    xs, ys = [], []
    for c in range(b.shape[1]):
        x, y = oracle_ts(orc, L, A, b[:, c])
        xs.append(x)
        ys.append(y)
    return np.stack(xs, 1), np.stack(ys, 1)


def test_s1_lap2d5_64_fp64(orc):
    announce("ts fused lap2d5_64 fp64")
    L, A = synth.workload("lap2d5_64")
    b = synth.vec_uniform(L.nrows, seed=1)
    s = sfm.Schedule(L, A)
    x, y = run(s, L, A, b)
    xr, yr = oracle_ts(orc, L, A, b)
    assert relerr(x, xr) <= TOL64 and relerr(y, yr) <= TOL64


@pytest.mark.parametrize("case", ["lap2d5_64", "random", "spd", "multi"])
def test_fp64_bit_identical_to_oracle(orc, case):
    """Each row subtracts the rounded products L_ij x_j from b_i in ascending
    column order and divides by L_ii, like the sequential definition, so the
    fused and unfused FP64 results equal the oracle's bit for bit."""
    announce("ts bit-identical " + case)
    if case == "lap2d5_64":
        L, A = synth.workload("lap2d5_64")
    elif case == "random":
        L = synth.random_lower(5003, 0.002, seed=11)
        A = synth.from_scipy(sp.random(2500, 5003, density=0.003, random_state=np.random.default_rng(3),
                                       format="csr"))
    else:
        A = synth.random_spd(30000, seed=5)
        L = synth.lower(A)
    k = 5 if case == "multi" else None
    b = synth.vec_uniform(L.nrows, k=k or 1, seed=2)
    s = sfm.Schedule(L, A, rows_per_item=23)
    xr, yr = oracle_ts(orc, L, A, b)
    for unfused in (False, True):
        x, y = run(s, L, A, b, unfused=unfused)
        assert np.array_equal(x, xr), ("x", unfused)
        assert np.array_equal(y, yr), ("y", unfused)
    for delay in (2, 1 << 20):  # SpMV rows placed later in the claim order
        s.set_param("spmv_delay", delay)
        x, y = run(s, L, A, b)
        assert np.array_equal(x, xr) and np.array_equal(y, yr), delay


def test_integer_manufactured_solution_bit_exact():
    """Integer L, A and x_true: every partial sum is an exact integer and the
    divisions are exact, so the GPU result must equal x_true and A x_true in
    any summation order."""
    announce("ts fused integer manufactured lap2d5_64 + random int")
    L, A = synth.workload("lap2d5_64")
    xt = synth.int_vector(L.nrows, seed=7)
    b = L.to_scipy() @ xt
    s = sfm.Schedule(L, A)
    x, y = run(s, L, A, b)
    assert np.array_equal(x, xt)
    assert np.array_equal(y, A.to_scipy() @ xt)
    Li = synth.random_lower(3001, 0.003, seed=4, int_values=True)
    Ai = synth.from_scipy(sp.random(1500, 3001, density=0.004, random_state=np.random.default_rng(1),
                                    format="csr", data_rvs=lambda k: np.random.default_rng(2).integers(-3, 4, k)))
    xt = synth.int_vector(3001, seed=8)
    b = Li.to_scipy() @ xt
    for lanes in (2, 4, 8, 16, 32):
        s = sfm.Schedule(Li, Ai, lanes_per_row=lanes, rows_per_item=37)
        x, y = run(s, Li, Ai, b)
        assert np.array_equal(x, xt), lanes
        assert np.array_equal(y, Ai.to_scipy() @ xt), lanes


@pytest.mark.parametrize("seed,n,m,rows,gt,gs", [
    (0, 1000, 1000, 64, 4, 8), (1, 2049, 777, 13, 8, 4), (2, 4097, 5000, 1, 2, 32),
    (3, 10007, 333, 200, 16, 16), (4, 65, 1, 64, 32, 4)])
def test_random_ragged(orc, seed, n, m, rows, gt, gs):
    announce("ts fused random n=%d m=%d rows=%d gt=%d gs=%d" % (n, m, rows, gt, gs))
    L = synth.random_lower(n, min(0.5, 6.0 / n), seed=seed)
    rng = np.random.default_rng(seed)
    a = sp.random(m, n, density=min(1.0, 9.0 / n), random_state=rng, format="csr")
    a = sp.csr_matrix(a.toarray() * (np.arange(m) % 7 != 3)[:, None])  # some empty rows
    A = synth.from_scipy(a)
    b = synth.vec_uniform(n, seed=seed + 1)
    s = sfm.Schedule(L, A, rows_per_item=rows)
    s.set_param("lanes_trsv", gt)
    s.set_param("lanes_spmv", gs)
    x, y = run(s, L, A, b)
    xr, yr = oracle_ts(orc, L, A, b)
    assert relerr(x, xr) <= TOL64
    assert relerr(y, yr) <= TOL64
    xu, yu = run(s, L, A, b, unfused=True)
    assert relerr(xu, xr) <= TOL64 and relerr(yu, yr) <= TOL64


def test_fp32_within_rounding_bound(orc):
    """FP32 values, vectors and accumulation: the computed x satisfies the
    componentwise backward-error bound of substitution in FP32,
    |b - L x| <= gamma_m |L| |x| (u = 2^-24), with L and b rounded to FP32."""
    announce("ts fused fp32 random spd 20000")
    a = synth.random_spd(20000, seed=3)
    L = synth.lower(a)
    b = synth.vec_uniform(a.nrows, seed=1)
    s = sfm.Schedule(L, a)
    x, y = run(s, L, a, b, dtype="f32")
    L32 = L.to_scipy().astype(np.float32).astype(np.float64)
    b32 = b.astype(np.float32).astype(np.float64)
    m = int(np.diff(L.rowptr).max())
    u = 2.0 ** -24
    gam = m * u / (1 - m * u)
    r = np.abs(b32 - L32 @ x)
    assert np.all(r <= 2 * gam * (abs(L32) @ np.abs(x)) + 1e-30)
    xr, yr = oracle_ts(orc, L, a, b)
    print("fp32 relative error vs FP64 oracle: x %.2e y %.2e" % (relerr(x, xr), relerr(y, yr)))
    assert relerr(x, xr) < 1e-4


@pytest.mark.parametrize("k,kb", [(2, 0), (3, 2), (8, 8), (13, 8), (13, 16), (64, 64), (64, 16), (33, 32)])
def test_multi_rhs(orc, k, kb):
    announce("ts fused multi-rhs k=%d kb=%d" % (k, kb))
    L, A = synth.workload("lap2d5_64")
    b = synth.vec_uniform(L.nrows, k=k, seed=1)
    s = sfm.Schedule(L, A, rhs_block=kb)
    x, y = run(s, L, A, b)
    xr, yr = oracle_ts(orc, L, A, b)
    # every column folds its terms in the definition's order: bit-identical
    assert np.array_equal(x, xr) and np.array_equal(y, yr)
    xu, yu = run(s, L, A, b, unfused=True)
    assert np.array_equal(xu, xr) and np.array_equal(yu, yr)


@pytest.mark.parametrize("m,k,kb", [(2500, 13, 8), (7001, 64, 64), (7001, 3, 0)])
def test_multi_rhs_padded_ld_rectangular(orc, m, k, kb):
    """Column-major B, X and Y with leading dimensions past their rows, and
    A with fewer or more rows than L: the interleaved blocks are packed and
    unpacked through the leading dimensions, the padding rows are never
    written, and FP64 results equal the oracle's bit for bit."""
    announce("ts multi-rhs padded ld m=%d k=%d kb=%d" % (m, k, kb))
    import torch
    n = 5003
    L = synth.random_lower(n, 0.002, seed=11)
    A = synth.from_scipy(sp.random(m, n, density=0.003, random_state=np.random.default_rng(3), format="csr"))
    b = synth.vec_uniform(n, k=k, seed=4)
    xr, yr = oracle_ts(orc, L, A, b)
    s = sfm.Schedule(L, A, rhs_block=kb)
    Lv, Av = dev(L.val), dev(A.val)
    for unfused in (False, True):
        Bbuf = torch.full((k, n + 7), 3.0, dtype=torch.float64, device="cuda")
        Bbuf[:, :n] = torch.as_tensor(b.T, device="cuda")
        Xbuf = torch.full((k, n + 5), -7.0, dtype=torch.float64, device="cuda")
        Ybuf = torch.full((k, m + 9), -9.0, dtype=torch.float64, device="cuda")
        X, Y = sfm.trsv_spmv(s, Lv, Av, Bbuf.t()[:n], X=Xbuf.t()[:n], Y=Ybuf.t()[:m], unfused=unfused)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr), unfused
        assert bool((Xbuf[:, n:] == -7.0).all()) and bool((Ybuf[:, m:] == -9.0).all()), unfused


def test_multi_rhs_integer_bit_exact():
    announce("ts fused multi-rhs integer")
    L, A = synth.workload("lap2d5_64")
    xt = np.stack([synth.int_vector(L.nrows, seed=s) for s in range(12)], 1)
    b = L.to_scipy() @ xt
    for kb in (4, 8, 16):
        s = sfm.Schedule(L, A, rhs_block=kb)
        x, y = run(s, L, A, b)
        assert np.array_equal(x, xt) and np.array_equal(y, A.to_scipy() @ xt)


def test_repeated_launches_and_modes(orc):
    """Epoch-tagged flags: many launches of one schedule (fused, unfused,
    solve only, multi-RHS) interleaved, each result exact."""
    announce("ts repeated launches")
    import torch
    L, A = synth.workload("lap2d5_64")
    xt = synth.int_vector(L.nrows, seed=3)
    b = L.to_scipy() @ xt
    yt = A.to_scipy() @ xt
    s = sfm.Schedule(L, A)
    Lv, Av, B = dev(L.val), dev(A.val), dev(b)
    for it in range(12):
        if it % 3 == 0:
            X, Y = sfm.trsv_spmv(s, Lv, Av, B)
        elif it % 3 == 1:
            X, Y = sfm.trsv_spmv(s, Lv, Av, B, unfused=True)
        else:
            X, Y = sfm.trsv_spmv(s, Lv, Av, B, want_y=False)
        torch.cuda.synchronize()
        assert np.array_equal(host(X), xt), it
        if Y is not None:
            assert np.array_equal(host(Y), yt), it
    Bk = dev_colmajor(np.stack([b, 2 * b, -b], 1))
    X, Y = sfm.trsv_spmv(s, Lv, Av, Bk)
    assert np.array_equal(host(X), np.stack([xt, 2 * xt, -xt], 1))
    sfm.sync_status(s)


def test_degenerate(orc):
    announce("ts degenerate n=1 and diagonal")
    L = synth.from_scipy(sp.csr_matrix(np.array([[2.0]])))
    A = synth.from_scipy(sp.csr_matrix(np.array([[3.0], [0.0]])))
    s = sfm.Schedule(L, A)
    x, y = run(s, L, A, np.array([5.0]))
    assert x.tolist() == [2.5] and y.tolist() == [7.5, 0.0]
    d = synth.from_scipy(sp.diags(np.arange(1.0, 301.0), format="csr"))
    s = sfm.Schedule(d, d)
    b = synth.vec_uniform(300, seed=2)
    x, y = run(s, d, d, b)
    assert np.array_equal(x, b / np.arange(1.0, 301.0))


def test_empty_system_zeroes_y():
    """No unknowns: x is empty and y = A x is zero for an A with rows but no
    columns.  Y starts as NaN and must come back zero from every entry: fused,
    unfused, three right-hand sides with a padded leading dimension, both
    static plans; an A without rows leaves nothing to write."""
    announce("ts empty system n=0 (m=5 and m=0)")
    import torch
    L = synth.from_scipy(sp.csr_matrix((0, 0)))
    A = synth.from_scipy(sp.csr_matrix((5, 0)))
    s = sfm.Schedule(L, A)
    Lv = torch.empty(0, dtype=torch.float64, device="cuda")
    for unfused in (False, True):
        Y = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        X, Y = sfm.trsv_spmv(s, Lv, None, torch.empty(0, dtype=torch.float64, device="cuda"), Y=Y,
                             unfused=unfused)
        torch.cuda.synchronize()
        assert X.shape == (0,) and host(Y).tolist() == [0.0] * 5, unfused
    big = torch.full((3, 8), float("nan"), dtype=torch.float32, device="cuda")
    Yk = big.t()[:5]                      # column-major (5, 3), leading dimension 8
    B = sfm.colmajor(0, 3, torch.float32)
    sfm.trsv_spmv(s, Lv.float(), None, B, Y=Yk)
    torch.cuda.synchronize()
    got = host(big)
    assert (got[:, :5] == 0).all() and np.isnan(got[:, 5:]).all()  # padding rows untouched
    for plan in (sfm.SF_STATIC_MSP, sfm.SF_STATIC_WAVEFRONT):
        Y = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        _, Y = sfm.static_trsv_spmv(s, plan, Lv, None, torch.empty(0, dtype=torch.float64, device="cuda"), Y=Y)
        torch.cuda.synchronize()
        assert host(Y).tolist() == [0.0] * 5, plan
    s0 = sfm.Schedule(L, synth.from_scipy(sp.csr_matrix((0, 0))))
    X, Y = sfm.trsv_spmv(s0, Lv, None, torch.empty(0, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert X.numel() == 0 and Y.numel() == 0
    sfm.sync_status(s)


def test_watchdog_reports_timeout_and_recovers(orc):
    """A spin limit of one poll makes waits on not-yet-final rows give up:
    the launch drains, SF_ERR_TIMEOUT is reported, and the next launch with
    the default limit is exact again."""
    announce("ts watchdog (forced from host)")
    L, A = synth.workload("lap2d5_64")
    xt = synth.int_vector(L.nrows, seed=3)
    b = L.to_scipy() @ xt
    s = sfm.Schedule(L, A)
    default = s.get_param("spin_limit")
    s.set_param("spin_limit", 1)
    s.set_param("rows_per_item", 1)
    import torch
    Lv, Av, B = dev(L.val), dev(A.val), dev(b)
    hit = False
    for _ in range(5):
        sfm.trsv_spmv(s, Lv, Av, B)
        try:
            sfm.sync_status(s)
        except sfm.SparseFusionError as e:
            assert e.name == "SF_ERR_TIMEOUT"
            hit = True
            break
    assert hit, "a one-poll watchdog never fired on a 127-level DAG"
    s.set_param("spin_limit", default)
    X, Y = sfm.trsv_spmv(s, Lv, Av, B)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    assert np.array_equal(host(X), xt)


def test_watchdog_timeout_stays_in_its_launch(orc):
    """A launch whose waits gave up does not shorten the waits of the next
    launch on the same schedule (each launch has its own status word), while
    the timeout is still reported by sf_sync_status afterwards (sticky)."""
    announce("ts watchdog: timed-out launches then an exact one, no sync between")
    L, A = synth.workload("lap2d5_64")
    xt = synth.int_vector(L.nrows, seed=3)
    b = L.to_scipy() @ xt
    s = sfm.Schedule(L, A)
    default = s.get_param("spin_limit")
    s.set_param("rows_per_item", 1)
    import torch
    Lv, Av, B = dev(L.val), dev(A.val), dev(b)
    s.set_param("spin_limit", 1)
    for _ in range(5):
        sfm.trsv_spmv(s, Lv, Av, B)
    s.set_param("spin_limit", default)
    X, Y = sfm.trsv_spmv(s, Lv, Av, B)
    torch.cuda.synchronize()
    assert np.array_equal(host(X), xt)
    with pytest.raises(sfm.SparseFusionError) as e:
        sfm.sync_status(s)
    assert e.value.name == "SF_ERR_TIMEOUT"
    sfm.sync_status(s)  # reported once, then clear


def _coarsened_case(case):
    if case == "lap3d7_20":
        A = synth.laplacian_3d7(20, 20, 20, 6.0)
    elif case == "lap2d9_64":
        A = synth.laplacian_2d9(64, 64, 8.0)
    elif case == "lap3d27_10":
        A = synth.laplacian_3d27(10, 10, 10, 26.1)
    elif case == "tridiag":
        A = synth.laplacian_1d(700, 2.0)
    elif case == "random":
        A = synth.random_spd(20000, seed=4)
    else:
        return synth.workload("lap2d5_64")
    return synth.lower(A), A


@pytest.mark.parametrize("case", ["lap3d7_20", "lap2d9_64", "lap3d27_10", "tridiag", "random", "lap2d5_64"])
def test_coarsened_bit_identical(orc, case):
    """Coarsened items (rows of several wavefronts in one item, the item's
    own x values kept in LDS) run the definition's arithmetic in its order:
    FP64 x and y equal the oracle's bit for bit, with full and small items,
    a tight cost budget and late SpMV rows.  The same schedule's multi-RHS and
    unfused paths (level items) stay exact too."""
    announce("ts coarsened bit-identical " + case)
    L, A = _coarsened_case(case)
    b = synth.vec_uniform(L.nrows, seed=2)
    xr, yr = oracle_ts(orc, L, A, b)
    for rows, budget, delay in ((64, 512, 0), (13, 40, 0), (64, 512, 2), (64, 512, 1 << 20)):
        s = sfm.Schedule(L, A, rows_per_item=rows, max_item_nnz=budget, coarsen=2)
        if delay:
            s.set_param("spmv_delay", delay)
        assert s.info().coarsened == 1
        x, y = run(s, L, A, b)
        assert np.array_equal(x, xr) and np.array_equal(y, yr), (rows, budget, delay)
    x, y = run(s, L, A, b, unfused=True)
    assert np.array_equal(x, xr) and np.array_equal(y, yr)
    b3 = synth.vec_uniform(L.nrows, k=3, seed=5)
    x3r, y3r = oracle_ts(orc, L, A, b3)
    x3, y3 = run(s, L, A, b3)
    assert np.array_equal(x3, x3r) and np.array_equal(y3, y3r)
    # SpTRSV alone (no A product) through the coarsened items
    import torch
    X, _ = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b), want_y=False)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    assert np.array_equal(host(X), xr)


def test_coarsened_integer_and_fp32(orc):
    """Integer manufactured solution through coarsened items (exact), and the
    FP32 coarsened solve within the same bound as level items."""
    announce("ts coarsened integer + fp32")
    A = synth.laplacian_3d7(16, 16, 16, 6.0)
    L = synth.lower(A)
    # same pattern, integer values: 1 on the diagonal, -1 off it
    Li = synth.from_scipy(sp.csr_matrix((np.where(L.col == np.repeat(np.arange(L.nrows), np.diff(L.rowptr)), 1.0, -1.0),
                                         L.col, L.rowptr), shape=(L.nrows, L.nrows)))
    xt = synth.int_vector(L.nrows, seed=3)
    b = Li.to_scipy() @ xt
    s = sfm.Schedule(Li, A, coarsen=2)
    x, _ = run(s, Li, A, b)
    assert np.array_equal(x, xt)
    bf = synth.vec_uniform(L.nrows, seed=1)
    xr, yr = oracle_ts(orc, L, A, bf)
    s = sfm.Schedule(L, A, coarsen=2)
    x32, y32 = run(s, L, A, bf, dtype="f32")
    s1 = sfm.Schedule(L, A, coarsen=1)
    x32l, y32l = run(s1, L, A, bf, dtype="f32")
    assert np.array_equal(x32, x32l) and np.array_equal(y32, y32l)  # same FP32 operations in the same order


@pytest.mark.parametrize("coarsen", [1, 2])
def test_long_rows_bit_exact(orc, coarsen):
    """Rows longer than one stream pass (512 entries): a few dense SpTRSV rows
    (one reading every earlier row) and dense SpMV rows among short ones, so
    items take several passes and coarsened plans keep such rows apart."""
    announce("ts long rows coarsen=%d" % coarsen)
    n = 3000
    rng = np.random.default_rng(21)
    L = sp.lil_matrix(sp.random(n, n, density=2.0 / n, random_state=rng, format="csr"))
    L = sp.tril(L, -1).tolil()
    for r in (1500, 2999):
        L[r, :r] = rng.uniform(-1, 1, r) / r
    L = (sp.tril(L, -1) + sp.diags(rng.uniform(1, 2, n))).tocsr()
    A = sp.random(n + 7, n, density=3.0 / n, random_state=rng, format="lil")
    A[5, :] = rng.uniform(-1, 1, n)
    A[n + 6, : n // 2] = rng.uniform(-1, 1, n // 2)
    Ls, As = synth.from_scipy(L), synth.from_scipy(A.tocsr())
    b = synth.vec_uniform(n, seed=3)
    xr, yr = oracle_ts(orc, Ls, As, b)
    for rows, budget in ((64, 512), (5, 100)):
        s = sfm.Schedule(Ls, As, coarsen=coarsen, rows_per_item=rows, max_item_nnz=budget)
        x, y = run(s, Ls, As, b)
        assert np.array_equal(x, xr) and np.array_equal(y, yr), (rows, budget)
    xu, yu = run(s, Ls, As, b, unfused=True)
    assert np.array_equal(xu, xr) and np.array_equal(yu, yr)


@pytest.mark.parametrize("coarsen", [1, 2])
def test_alternating_rhs_bit_exact(orc, coarsen):
    """Launches that alternate right-hand sides on one schedule: each result
    equals the oracle's for its own b, so no value of an earlier launch is
    ever taken for a final one (first reads of x go through the caches)."""
    announce("ts alternating rhs coarsen=%d" % coarsen)
    import torch
    A = synth.laplacian_3d7(24, 24, 24, 6.0)
    L = synth.lower(A)
    bs = [synth.vec_uniform(L.nrows, seed=s) for s in (11, 12, 13)]
    refs = [oracle_ts(orc, L, A, b) for b in bs]
    s = sfm.Schedule(L, A, coarsen=coarsen)
    Lv, Av = dev(L.val), dev(A.val)
    Bs = [dev(b) for b in bs]
    X = torch.empty(L.nrows, dtype=torch.float64, device="cuda")
    Y = torch.empty(A.nrows, dtype=torch.float64, device="cuda")
    for it in range(12):
        k = it % 3
        sfm.trsv_spmv(s, Lv, Av, Bs[k], X=X, Y=Y)
        torch.cuda.synchronize()
        assert np.array_equal(host(X), refs[k][0]) and np.array_equal(host(Y), refs[k][1]), it
    sfm.sync_status(s)


@pytest.mark.parametrize("name", ["lap3d7_128", "randspd_1m"])
def test_full_size_configs(orc, name):
    """The benchmark's workloads at full size, whole vectors against the
    oracle (bit-identical in FP64), with the plan the inspector chose."""
    announce("ts fused full size " + name)
    L, A = synth.workload(name)
    b = synth.vec_uniform(L.nrows, seed=1)
    s = sfm.Schedule(L, A)
    x, y = run(s, L, A, b)
    xr, yr = oracle_ts(orc, L, A, b)
    ex, ey = relerr(x, xr), relerr(y, yr)
    print("%s fused (coarsened=%d): x err %.2e  y err %.2e" % (name, s.info().coarsened, ex, ey))
    assert ex <= TOL64 and ey <= TOL64
    assert np.array_equal(x, xr) and np.array_equal(y, yr)
    xu, yu = run(s, L, A, b, unfused=True)
    assert relerr(xu, xr) <= TOL64 and relerr(yu, yr) <= TOL64


@pytest.mark.parametrize("kb", [8, 64])
def test_multi_rhs_alternating_bit_exact(orc, kb):
    """Launches with different right-hand sides in turn, fused and unfused,
    on one schedule (whose interleaved workspace is reused at the same
    address): every result is exact, so no value of an earlier launch is
    ever taken for a published one."""
    announce("ts multi-rhs alternating kb=%d" % kb)
    import torch
    L, A = synth.workload("lap2d5_64")
    Ls, As = L.to_scipy(), A.to_scipy()
    sets = []
    for t in range(3):
        xt = np.stack([synth.int_vector(L.nrows, seed=10 * t + c) for c in range(kb)], 1)
        sets.append((dev_colmajor(Ls @ xt), xt, As @ xt))
    s = sfm.Schedule(L, A, rhs_block=kb)
    Lv, Av = dev(L.val), dev(A.val)
    for it in range(9):
        B, xt, yt = sets[it % 3]
        X, Y = sfm.trsv_spmv(s, Lv, Av, B, unfused=(it % 4 == 3))
        torch.cuda.synchronize()
        assert np.array_equal(host(X), xt) and np.array_equal(host(Y), yt), it
    sfm.sync_status(s)


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("coarsen", [1, 2])
def test_multi_rhs_paths_bit_exact(orc, path, coarsen):
    """Several right-hand sides through either path -- interleaved blocks over
    the level units, or one chain of the single-RHS items per column on the
    caller's columns -- on level and coarsened plans, with leading
    dimensions past the rows: FP64 results equal the oracle's bit for bit
    and the padding rows are never written."""
    announce("ts multi-rhs path=%d coarsen=%d" % (path, coarsen))
    import torch
    n, k = 5003, 11
    L = synth.random_lower(n, 0.002, seed=11)
    A = synth.from_scipy(sp.random(4000, n, density=0.003, random_state=np.random.default_rng(3), format="csr"))
    b = synth.vec_uniform(n, k=k, seed=6)
    xr, yr = oracle_ts(orc, L, A, b)
    s = sfm.Schedule(L, A, coarsen=coarsen)
    s.set_param("multi_path", path)
    assert s.get_param("multi_path") == path
    Lv, Av = dev(L.val), dev(A.val)
    for unfused in (False, True):
        Bbuf = torch.full((k, n + 3), 5.0, dtype=torch.float64, device="cuda")
        Bbuf[:, :n] = torch.as_tensor(b.T, device="cuda")
        Xbuf = torch.full((k, n + 6), -7.0, dtype=torch.float64, device="cuda")
        Ybuf = torch.full((k, 4000 + 2), -9.0, dtype=torch.float64, device="cuda")
        X, Y = sfm.trsv_spmv(s, Lv, Av, Bbuf.t()[:n], X=Xbuf.t()[:n], Y=Ybuf.t()[:4000], unfused=unfused)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr), unfused
        assert bool((Xbuf[:, n:] == -7.0).all()) and bool((Ybuf[:, 4000:] == -9.0).all()), unfused


@pytest.mark.parametrize("case", ["spd", "partial", "spd_f32", "chains"])
def test_prefix_fusion(orc, case):
    """Prefix fusion on level items: SpMV row r's entries up to its diagonal
    (their columns exactly L's row r) are folded by SpTRSV row r's item from
    the x values it gathers, and the SpMV row continues the fold from that
    partial sum -- A's entry order kept, so y equals the oracle's ordered
    fold bit for bit, with the prefix on and off.  "partial": L misses some
    of lower(A)'s entries, so only some rows qualify; "chains": three
    right-hand sides as column chains of the level items."""
    import torch
    announce("ts prefix fusion " + case)
    A = synth.random_spd(30000, seed=7)
    L = synth.lower(A)
    if case == "partial":
        Ls = L.to_scipy().tocoo()
        keep = (Ls.row == Ls.col) | (np.random.default_rng(4).random(Ls.nnz) < 0.7)
        L = synth.from_scipy(sp.csr_matrix((Ls.data[keep], (Ls.row[keep], Ls.col[keep])), shape=Ls.shape))
    k = 3 if case == "chains" else None
    b = synth.vec_uniform(L.nrows, k=k or 1, seed=9)
    s = sfm.Schedule(L, A, coarsen=1)
    rows = s.get_param("prefix_rows")
    if case == "partial":
        assert 0 < rows < L.nrows
    else:
        assert rows == L.nrows
    if case == "chains":
        s.set_param("multi_path", 2)
    dt = "f32" if case == "spd_f32" else "f64"
    assert s.get_param("spmv_prefix") == 1
    x1, y1 = run(s, L, A, b, dtype=dt)
    s.set_param("spmv_prefix", 0)
    x0, y0 = run(s, L, A, b, dtype=dt)
    assert np.array_equal(x1, x0) and np.array_equal(y1, y0)
    if dt == "f64":
        xr, yr = oracle_ts(orc, L, A, b)
        assert np.array_equal(x1, xr) and np.array_equal(y1, yr)
    s.set_param("spmv_prefix", 1)
    s.set_param("spmv_delay", 1 << 20)  # SpMV rows after every SpTRSV row
    x2, y2 = run(s, L, A, b, dtype=dt)
    assert np.array_equal(x2, x0) and np.array_equal(y2, y0)


@pytest.mark.parametrize("scale", [1, 2, 4, 8])
def test_spmv_item_scale_bit_identical(orc, scale):
    """Larger SpMV items on level items (spmv_item_scale) change only which
    rows a wavefront claims together, never a row's terms or their order:
    x and y equal the oracle's, with prefix fusion on and off."""
    announce("ts spmv_item_scale %d" % scale)
    A = synth.random_spd(30000, seed=11)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, seed=3)
    s = sfm.Schedule(L, A, coarsen=1, rows_per_item=16)
    s.set_param("spmv_item_scale", scale)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    yr = orc.spmv(A.rowptr, A.col, A.val, xr)
    for prefix in (1, 0):
        s.set_param("spmv_prefix", prefix)
        x, y = run(s, L, A, b)
        assert np.array_equal(x, xr) and np.array_equal(y, yr), prefix
