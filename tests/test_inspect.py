"""Host inspector (sf_inspect) against the oracle: levels, joint order,
items, reversed levels and structural errors.  Host only, no GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth

CASES = ["lap2d5_16", "lap2d5_64"]


def _random_pair(n, seed, m=None, empty_rows=False):
    L = synth.random_lower(n, 0.01 if n > 500 else 0.1, seed=seed)
    m = n if m is None else m
    rng = np.random.default_rng(seed + 100)
    a = sp.random(m, n, density=min(1.0, 8.0 / n), random_state=rng, format="csr")
    if empty_rows:
        a = sp.csr_matrix(a.toarray() * (np.arange(m) % 5 != 0)[:, None])
    return L, synth.from_scipy(a)


def _check_schedule(orc, L, A, s):
    level, order, item_ptr = s.export()
    lv, depth = orc.levels(L.rowptr, L.col)
    assert np.array_equal(level, lv), "levels differ from the oracle"
    st = s.info()
    assert st.depth == depth
    ready = orc.spmv_ready(A.rowptr, A.col, lv)
    want = orc.joint_order_ts(lv, ready)
    assert np.array_equal(order, want), "claim order differs from the canonical joint order"
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, item_ptr) == 0
    assert st.joint_depth == max(depth, int(ready.max()) + 1 if len(ready) else 0)
    widths = np.bincount(lv)
    assert st.max_level_width == widths.max()


@pytest.mark.parametrize("name", CASES)
def test_stencil_schedules(orc, name):
    L, A = synth.workload(name)
    s = sfm.Schedule(L, A, validate=True, coarsen=1)
    _check_schedule(orc, L, A, s)
    assert abs(s.info().reuse_ratio - orc.reuse_ts(L.nrows, L.nnz, A.nrows, A.nnz)) < 1e-15


@pytest.mark.parametrize("seed,n,m,empty", [(0, 60, None, False), (1, 1000, None, True), (2, 777, 300, True),
                                              (3, 500, 900, False)])
def test_random_schedules(orc, seed, n, m, empty):
    L, A = _random_pair(n, seed, m, empty)
    for rows in (1, 7, 64):
        s = sfm.Schedule(L, A, rows_per_item=rows, max_item_nnz=50, validate=True, coarsen=1)
        for scale in (s.get_param("spmv_item_scale"), 1):
            s.set_param("spmv_item_scale", scale)
            _check_schedule(orc, L, A, s)
            _, order, ip = s.export()
            sizes = np.diff(ip)
            spmv = order[ip[:-1]] >= L.nrows
            # SpTRSV items hold at most rows_per_item rows, SpMV items (off
            # the critical path) up to spmv_item_scale times that, at most 64
            assert sizes[~spmv].max(initial=0) <= rows
            assert sizes[spmv].max(initial=0) <= min(64, rows * scale)


@pytest.mark.parametrize("delay", [1, 3, 1000])
def test_spmv_delay_orders_stay_valid(orc, delay):
    """SpMV rows are slack iterations: placing them `delay` wavefronts after
    their joint level keeps every DAG edge respected (the oracle's
    validator), keeps the SpTRSV rows in canonical order, and puts no SpMV row
    before its joint level."""
    for L, A in (synth.workload("lap2d5_64"), _random_pair(1500, 7, 900, True)):
        s = sfm.Schedule(L, A, rows_per_item=20, validate=True, coarsen=1)
        s.set_param("spmv_delay", delay)
        level, order, ip = s.export()
        assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, ip) == 0
        n = L.nrows
        trsv = order[order < n]
        assert np.array_equal(trsv, np.lexsort((np.arange(n), level)))
        ready = orc.spmv_ready(A.rowptr, A.col, level)
        pos = np.empty(len(order), int)
        pos[order] = np.arange(len(order))
        # the SpTRSV rows of level ready + delay (when that level exists) come before it
        for r in range(0, A.nrows, 37):
            want_after = np.nonzero(level == min(ready[r] + delay, level.max()))[0]
            if ready[r] + delay <= level.max() and len(want_after):
                assert pos[n + r] > pos[want_after].max()
        s.set_param("spmv_delay", 0)
        assert np.array_equal(s.export()[1], orc.joint_order_ts(level, ready))


def _check_coarsened(orc, L, A, s):
    """A coarsened plan: every DAG edge respected (the oracle's validator,
    edges inside an item allowed), each item's rows sorted by local
    wavefront, every edge inside an item going to a later local wavefront,
    and the per-entry slots naming exactly the item-local columns."""
    level, order, ip = s.export()
    loc, slot = s.export_local()
    n = L.nrows
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, ip, allow_intra=True) == 0
    item = np.repeat(np.arange(len(ip) - 1), np.diff(ip))
    pos = np.empty(len(order), np.int64)
    pos[order] = np.arange(len(order))
    for t in range(len(ip) - 1):
        seg = loc[ip[t]:ip[t + 1]]
        assert np.all(np.diff(seg.astype(int)) >= 0)
        if order[ip[t]] >= n:
            assert not seg.any()  # SpMV items hold independent rows
        else:
            assert np.all(order[ip[t]:ip[t + 1]] < n)  # items are kind-pure
            assert ip[t + 1] - ip[t] <= 64
    rows = np.repeat(np.arange(n), np.diff(L.rowptr))
    off = L.col != rows
    u, v, pslot = L.col[off], rows[off], slot[off]
    same = item[pos[u]] == item[pos[v]]
    assert np.all(loc[pos[u][same]] < loc[pos[v][same]])
    assert np.array_equal(pslot[same].astype(np.int64), pos[u][same] - ip[item[pos[v][same]]])
    assert np.all(pslot[~same] == 255)
    # one stream pass per coarsened item
    for t in range(len(ip) - 1):
        if order[ip[t]] < n and loc[ip[t + 1] - 1] > 0:
            r = order[ip[t]:ip[t + 1]]
            assert int(np.sum(np.diff(L.rowptr)[r] - 1)) <= 512


@pytest.mark.parametrize("case", ["lap3d7_20", "lap2d9_64", "lap3d27_10", "random", "random_rect", "tridiag"])
def test_coarsened_plans(orc, case):
    if case == "lap3d7_20":
        A = synth.laplacian_3d7(20, 20, 20, 6.0)
        L = synth.lower(A)
    elif case == "lap2d9_64":
        A = synth.laplacian_2d9(64, 64, 8.0)
        L = synth.lower(A)
    elif case == "lap3d27_10":
        A = synth.laplacian_3d27(10, 10, 10, 26.1)
        L = synth.lower(A)
    elif case == "random":
        L, A = _random_pair(3000, 5, None, True)
    elif case == "random_rect":
        L, A = _random_pair(777, 6, 1300, True)
    else:
        A = synth.laplacian_1d(500, 2.0)
        L = synth.lower(A)
    for rows, budget, delay in ((64, 512, 0), (17, 40, 0), (64, 512, 3)):
        s = sfm.Schedule(L, A, rows_per_item=rows, max_item_nnz=budget, coarsen=2, validate=True)
        if delay:
            s.set_param("spmv_delay", delay)
        st = s.info()
        assert st.coarsened == 1 and st.chunk_items > 0
        _check_coarsened(orc, L, A, s)
        _, _, ip = s.export()
        assert np.diff(ip).max() <= rows
    if case == "tridiag":
        # a chain: every item is a run of consecutive rows, one wavefront each
        s = sfm.Schedule(L, A, coarsen=2)
        assert s.info().chunk_chain == (500 + 63) // 64 and s.info().max_local_depth == 64


def test_coarsen_choice():
    """The inspector keeps coarsened items where its critical-path estimate
    is clearly lower (mesh-like DAGs) and level items otherwise."""
    A = synth.laplacian_3d7(24, 24, 24, 6.0)
    s = sfm.Schedule(synth.lower(A), A)
    st = s.info()
    assert st.coarsened == 1 and st.est_chunk_us < 0.8 * st.est_level_us
    assert st.chunk_chain < st.depth
    # and the region plan over them where its estimate is lower still
    assert s.get_param("regioned") == 1
    L, A = _random_pair(5000, 9)
    assert sfm.Schedule(L, A).get_param("regioned") == 0
    st = sfm.Schedule(L, A).info()
    assert st.coarsened == 0 and (st.chunk_items == 0 or st.est_chunk_us >= 0.8 * st.est_level_us)
    Ar = synth.random_spd(20000, seed=1)  # edges skip many wavefronts: not even estimated
    st = sfm.Schedule(synth.lower(Ar), Ar).info()
    assert st.coarsened == 0 and st.chunk_items == 0
    st = sfm.Schedule(L, A, coarsen=1).info()
    assert st.coarsened == 0 and st.chunk_items == 0
    s = sfm.Schedule(L, A, coarsen=2)
    assert s.info().coarsened == 1
    s.set_param("coarsen", 1)
    assert s.info().coarsened == 0 and s.get_param("coarsened") == 0


def test_item_nnz_budget():
    L, A = synth.workload("lap2d5_64")
    s = sfm.Schedule(L, A, rows_per_item=1000, max_item_nnz=40, coarsen=1)
    scale = s.get_param("spmv_item_scale")
    assert scale == 4
    level, order, ip = s.export()
    n = L.nrows
    # cost c(v) = entries an iteration streams (SpTRSV: off-diagonals; at least 1);
    # SpMV items get spmv_item_scale times the budget
    cost = np.concatenate([np.maximum(1, np.diff(L.rowptr) - 1), np.maximum(1, np.diff(A.rowptr))])
    for t in range(len(ip) - 1):
        ids = order[ip[t]:ip[t + 1]]
        kinds = ids >= n
        assert kinds.all() or not kinds.any(), "an item mixes SpTRSV and SpMV rows"
        assert len(ids) == 1 or cost[ids].sum() <= (40 * scale if kinds.all() else 40)


def test_backward_schedule(orc):
    L, A = synth.workload("lap2d5_16")
    s = sfm.Schedule(L, A, want_backward=True, coarsen=1)
    rl, order, ip = s.export_backward()
    want, depth = orc.reverse_levels(L.rowptr, L.col)
    assert np.array_equal(rl, want)
    assert s.info().back_depth == depth
    # rows sorted by (reversed level, row); items hold one reversed level
    assert np.array_equal(order, np.lexsort((np.arange(L.nrows), want)))
    for t in range(len(ip) - 1):
        assert len(set(rl[order[ip[t]:ip[t + 1]]])) == 1
    # every edge of the transposed solve (lambda_j -> lambda_i for L_ji, j > i)
    # points from an earlier item to a later one
    item = np.empty(L.nrows, int)
    for t in range(len(ip) - 1):
        item[order[ip[t]:ip[t + 1]]] = t
    rows = np.repeat(np.arange(L.nrows), np.diff(L.rowptr))
    off = L.col < rows
    assert np.all(item[rows[off]] < item[L.col[off]])


@pytest.mark.parametrize("case", ["lap3d7_16", "lap2d9_48", "random"])
def test_coarsened_backward_plan(orc, case):
    """The coarsened plan of the transposed solve: a permutation of the rows
    in which every edge lambda_j -> lambda_i (L_ji stored, j > i) goes to a
    later item or, inside an item, to a later local wavefront, with the
    per-entry slots of L^T naming exactly the item-local columns."""
    if case == "lap3d7_16":
        A = synth.laplacian_3d7(16, 16, 16, 6.0)
        L = synth.lower(A)
    elif case == "lap2d9_48":
        A = synth.laplacian_2d9(48, 48, 8.0)
        L = synth.lower(A)
    else:
        L, A = _random_pair(2000, 3)
    s = sfm.Schedule(L, A, want_backward=True, coarsen=2, validate=True)
    st = s.info()
    assert st.back_coarsened == 1
    rl, order, ip = s.export_backward()
    loc, slot = s.export_backward_local()
    want, depth = orc.reverse_levels(L.rowptr, L.col)
    assert np.array_equal(rl, want) and st.back_depth == depth
    n = L.nrows
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.diff(ip).max() <= 64
    item = np.repeat(np.arange(len(ip) - 1), np.diff(ip))
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    for t in range(len(ip) - 1):
        assert np.all(np.diff(loc[ip[t]:ip[t + 1]].astype(int)) >= 0)
    # L^T in CSR: row i holds i (diagonal first) then the rows j > i with L_ji stored
    lt = L.to_scipy().T.tocsr()
    lt.sort_indices()
    rows = np.repeat(np.arange(n), np.diff(lt.indptr))
    j = lt.indices
    assert np.all(j[lt.indptr[:-1]] == np.arange(n))  # diagonal first
    off = j != rows
    u, v, ps = j[off], rows[off], slot[off]           # edge lambda_u -> lambda_v
    same = item[pos[u]] == item[pos[v]]
    assert np.all(item[pos[u]][~same] < item[pos[v]][~same])
    assert np.all(loc[pos[u][same]] < loc[pos[v][same]])
    assert np.array_equal(ps[same].astype(np.int64), pos[u][same] - ip[item[pos[v][same]]])
    assert np.all(ps[~same] == 255) and np.all(slot[~off] == 255)


def test_ic0_schedule(orc):
    a = synth.laplacian_3d27(6, 5, 4, 26.1)
    L = synth.lower(a)
    s = sfm.Schedule(L, None, sfm.SF_IC0_TRSV, validate=True)
    level, order, ip = s.export()
    lv, depth = orc.levels(L.rowptr, L.col)
    assert np.array_equal(level, lv)
    n = L.nrows
    assert sorted(order.tolist()) == list(range(2 * n))
    # each row's SpIC0 iteration directly precedes its SpTRSV iteration, in one item
    assert np.array_equal(order[1::2], order[0::2] + n)
    item = np.empty(2 * n, int)
    for t in range(len(ip) - 1):
        assert (ip[t + 1] - ip[t]) % 2 == 0
        item[order[ip[t]:ip[t + 1]]] = t
    rows = np.repeat(np.arange(n), np.diff(L.rowptr))
    off = L.col < rows
    assert np.all(item[L.col[off]] < item[rows[off]])            # SpIC0 j -> SpIC0 i
    assert np.all(item[n + L.col[off]] < item[n + rows[off]])    # SpTRSV j -> SpTRSV i
    assert abs(s.info().reuse_ratio - orc.reuse_it(n, L.nnz)) < 1e-15
    assert s.info().reuse_ratio >= 1.0
    assert orc.validate_factor_solve(L.rowptr, L.col, order, ip) == 0


@pytest.mark.parametrize("case", ["lap3d27_8", "lap3d27_8_perm", "random_spd", "lanes_4", "lanes_64"])
def test_factor_solve_schedules_oracle_valid(orc, case):
    """Every SpIC0 -> SpTRSV and SpILU0 -> SpTRSV schedule the inspector
    produces passes the oracle's factor -> solve check (every dependence to a
    later item, each row's solve after its factor row in the same item), at
    every lanes-per-row setting; the canonical levels equal the oracle's."""
    if case.startswith("lap3d27"):
        a = synth.laplacian_3d27(8, 8, 8, 26.1)
        if case.endswith("perm"):
            a = synth.permute_sym(a, synth.permutation(a.nrows, seed=3))
    elif case == "random_spd":
        a = synth.random_spd(3000, seed=4, lo=2, hi=6)
    else:
        a = synth.laplacian_3d27(6, 7, 5, 26.1)
    L = synth.lower(a)
    lanes = {"lanes_4": 4, "lanes_64": 64}.get(case, 0)
    s = sfm.Schedule(L, None, sfm.SF_IC0_TRSV, lanes_per_row=lanes)
    level, order, ip = s.export()
    assert np.array_equal(level, orc.levels(L.rowptr, L.col)[0])
    assert orc.validate_factor_solve(L.rowptr, L.col, order, ip) == 0
    # the same pattern as a (symmetric) SpILU0 input, whole matrix
    s2 = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV, lanes_per_row=max(lanes, 32) if lanes else 0)
    _, order2, ip2 = s2.export()
    assert orc.validate_factor_solve(a.rowptr, a.col, order2, ip2) == 0


def _err(fn):
    with pytest.raises(sfm.SparseFusionError) as e:
        fn()
    return e.value.name


def test_structural_errors():
    L, A = synth.workload("lap2d5_16")
    bad = L.col.copy()
    bad[[1, 2]] = bad[[2, 1]]  # row 1 unsorted (two entries)
    assert _err(lambda: sfm.Schedule((L.rowptr, bad, L.ncols), A)) == "SF_ERR_CSR"
    dup = L.col.copy()
    dup[2] = dup[1]
    assert _err(lambda: sfm.Schedule((L.rowptr, dup, L.ncols), A)) == "SF_ERR_CSR"
    oor = L.col.copy()
    oor[0] = L.ncols
    assert _err(lambda: sfm.Schedule((L.rowptr, oor, L.ncols), A)) == "SF_ERR_CSR"
    # A itself (has upper entries) given as L
    assert _err(lambda: sfm.Schedule(A, A)) == "SF_ERR_NOT_LOWER"
    # strictly lower part only: no diagonal
    sl = synth.from_scipy(sp.tril(L.to_scipy(), k=-1) + sp.csr_matrix((L.nrows, L.nrows)))
    nodiag_rp = np.concatenate([[0], np.cumsum(np.diff(sl.rowptr))]).astype(np.int32)
    assert _err(lambda: sfm.Schedule((nodiag_rp, sl.col, L.ncols), A)) == "SF_ERR_ZERO_DIAG"
    # A with the wrong number of columns
    assert _err(lambda: sfm.Schedule(L, (A.rowptr, A.col, A.ncols + 1))) == "SF_ERR_SHAPE"
    # decreasing row pointer
    rp = L.rowptr.copy()
    rp[5] = rp[6] + 1
    assert _err(lambda: sfm.Schedule((rp, L.col, L.ncols), A)) == "SF_ERR_CSR"
    # SpTRSV -> SpMV needs A
    assert _err(lambda: sfm.Schedule(L, None)) == "SF_ERR_ARG"


def test_degenerate_sizes(orc):
    # n = 0
    s = sfm.Schedule((np.zeros(1, np.int32), np.zeros(0, np.int32), 0), (np.zeros(1, np.int32), np.zeros(0, np.int32), 0))
    st = s.info()
    assert st.n == 0 and st.n_items == 0 and st.depth == 0
    # n = 1, A with one empty row and one full row
    L = (np.array([0, 1], np.int32), np.array([0], np.int32), 1)
    A = (np.array([0, 0, 1], np.int32), np.array([0], np.int32), 1)
    s = sfm.Schedule(L, A, validate=True, coarsen=1)
    level, order, ip = s.export()
    assert level.tolist() == [0]
    # empty SpMV row 0 has joint level 0 (after SpTRSV row 0 in the order), row 1 level 1
    assert order.tolist() == [0, 1, 2]
    assert s.info().joint_depth == 2
    # a diagonal L has one level
    d = synth.from_scipy(sp.identity(50, format="csr"))
    s = sfm.Schedule(d, d)
    assert s.info().depth == 1 and s.info().joint_depth == 2


def test_inspector_time_reported():
    L, A = synth.workload("lap2d5_64")
    s = sfm.Schedule(L, A, want_backward=True)
    assert 0.0 < s.info().inspect_seconds < 5.0


def test_ilu0_schedule(orc):
    """SpILU0 schedules: levels of the dependences left of the diagonal (the
    oracle's levels of the lower triangle), every dependence to a later item,
    one batch per item, and intersection lists equal to a brute-force count
    of the triples (k, j) with k < min(i, j) stored in row i and (k, j)
    stored in row k."""
    for a in (synth.convdiff_3d7(6, 5, 4), synth.random_nonsym(400, seed=3)):
        s = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV, validate=True)
        level, order, ip = s.export()
        low = synth.lower(a)
        lv, depth = orc.levels(low.rowptr, low.col)
        assert np.array_equal(level, lv) and s.info().depth == depth
        n = a.nrows
        rows = order[0::2]
        assert np.array_equal(order[1::2], rows + n)  # factor row i, then solve row i
        assert np.array_equal(np.sort(rows), np.arange(n))
        item = np.empty(n, int)
        for t in range(len(ip) - 1):
            item[order[ip[t]:ip[t + 1]:2]] = t
        r = np.repeat(np.arange(n), np.diff(a.rowptr))
        left = a.col < r
        assert np.all(item[a.col[left]] < item[r[left]])
        dense = a.to_scipy().toarray() != 0
        want = sum(int(np.sum(dense[i, :min(i, j)] & dense[:min(i, j), j]))
                   for i in range(n) for j in np.nonzero(dense[i])[0])
        st = s.info()
        assert st.lanes_per_row >= np.diff(a.rowptr).max()
        assert want == _ilu_pair_count(s)
        assert orc.validate_factor_solve(a.rowptr, a.col, order, ip) == 0


def _ilu_pair_count(s):
    # size of the schedule's intersection lists (read-only parameter)
    import ctypes
    lib = sfm._lib()
    v = ctypes.c_int64(0)
    assert lib.sf_get_param(s.handle, b"pairs", ctypes.byref(v)) == 0
    return int(v.value)


def test_ilu0_structural_errors():
    a = synth.convdiff_3d7(4, 4, 3)
    m = a.to_scipy().tolil()
    m[5, 5] = 0
    m = m.tocsr()
    m.eliminate_zeros()
    with pytest.raises(sfm.SparseFusionError) as e:
        sfm.Schedule(synth.from_scipy(m), None, sfm.SF_ILU0_TRSV)
    assert e.value.name == "SF_ERR_ZERO_DIAG"
    r = synth.from_scipy(sp.random(30, 40, density=0.2, random_state=1, format="csr"))
    with pytest.raises(sfm.SparseFusionError) as e:
        sfm.Schedule(r, None, sfm.SF_ILU0_TRSV)
    assert e.value.name == "SF_ERR_SHAPE"


def test_rhs_block_must_be_a_kernel_width():
    """The multi-RHS kernels exist for blocks of 2, 4, ..., 64 columns; other
    widths are refused at inspection and by set_param, never at launch."""
    L, A = synth.workload("lap2d5_16")
    for bad in (1, 3, 12, 65, -2):
        assert _err(lambda: sfm.Schedule(L, A, rhs_block=bad)) == "SF_ERR_ARG", bad
    for good in (0, 2, 8, 64):
        sfm.Schedule(L, A, rhs_block=good).free()
    s = sfm.Schedule(L, A)
    for bad in (1, 3, 128):
        assert _err(lambda: s.set_param("rhs_block", bad)) == "SF_ERR_ARG", bad
    s.set_param("rhs_block", 16)
    assert s.get_param("rhs_block") == 16


def _static_cases(name):
    import scipy.sparse as sp
    if name == "random":
        L = synth.random_lower(3001, 0.003, seed=5)
        A = synth.from_scipy(sp.random(2000, 3001, density=0.002, random_state=np.random.default_rng(2),
                                       format="csr"))
        return L, A
    if name == "chains":  # 8 independent bidiagonal chains of 50 rows
        blk = sp.diags([np.full(49, -1.0), np.full(50, 2.0)], [-1, 0])
        L = synth.from_scipy(sp.block_diag([blk] * 8, format="csr"))
        return L, synth.from_scipy(sp.identity(400, format="csr"))
    if name == "empty_rows":  # SpMV rows without entries
        L, A = synth.workload("lap2d5_16")
        a = A.to_scipy().tolil()
        a[3, :] = 0
        a[100, :] = 0
        return L, synth.from_scipy(a.tocsr())
    return synth.workload(name)


@pytest.mark.parametrize("case", ["lap2d5_64", "random", "chains", "empty_rows"])
def test_static_plans_respect_every_edge(orc, case):
    """Both static plans -- the paper's fused partitioning and the fused
    wavefront -- pass the oracle's two-level schedule check (every vertex
    once; every edge across s-partitions or in order inside one
    w-partition). The wavefront plan has one s-partition per wavefront of
    the joint DAG, w-partitions of at most 64 rows of one kind and level."""
    L, A = _static_cases(case)
    s = sfm.Schedule(L, A)
    n = L.nrows
    for plan in (sfm.SF_STATIC_MSP, sfm.SF_STATIC_WAVEFRONT):
        s_ptr, w_ptr, order = s.export_static(plan)
        assert orc.validate_static_ts(L.rowptr, L.col, A.rowptr, A.col, s_ptr, w_ptr, order) == 0, plan
    s_ptr, w_ptr, order = s.export_static(sfm.SF_STATIC_WAVEFRONT)
    lv, _ = orc.levels(L.rowptr, L.col)
    ready = orc.spmv_ready(A.rowptr, A.col, lv)
    joint = np.concatenate([lv, ready])
    assert len(s_ptr) - 1 == len(np.unique(joint))
    for w in range(len(w_ptr) - 1):
        ids = order[w_ptr[w]:w_ptr[w + 1]]
        assert 1 <= len(ids) <= 64 and len(np.unique(joint[ids])) == 1 and len(np.unique(ids < n)) == 1


def test_msp_windows_and_pairs(orc):
    """MSP on independent chains: every wavefront keeps the same 8
    components, so one window takes them all and each chain runs on one
    w-partition. Each chain's SpMV rows form its pair partition, and both
    sides have slack 0 (the chain is the critical path), so the merge step
    puts the pair after the chain in its w-partition: one s-partition, no
    barrier. With r = 1 the window puts all chains on one w-partition.
    On a 2D 5-point grid one more wavefront joins every piece, so each
    window is one wavefront (as many s-partitions as the level-set)."""
    L, A = _static_cases("chains")
    s = sfm.Schedule(L, A)
    s_ptr, w_ptr, order = s.export_static(sfm.SF_STATIC_MSP)
    assert len(s_ptr) - 1 == 1 and s.static_info(sfm.SF_STATIC_MSP)["merged"] == 8
    for w in range(s_ptr[0], s_ptr[1]):
        ids = order[w_ptr[w]:w_ptr[w + 1]]
        # one whole chain in order, then its SpMV rows in order
        c = ids[0] // 50
        want = np.concatenate([np.arange(50 * c, 50 * c + 50), 400 + np.arange(50 * c, 50 * c + 50)])
        assert np.array_equal(ids, want)
    s.set_param("msp_parts", 1)
    assert s.get_param("msp_parts") == 1
    s_ptr, w_ptr, order = s.export_static(sfm.SF_STATIC_MSP)
    assert s_ptr[1] - s_ptr[0] == 1
    assert orc.validate_static_ts(L.rowptr, L.col, A.rowptr, A.col, s_ptr, w_ptr, order) == 0
    L, A = synth.workload("lap2d5_64")
    s = sfm.Schedule(L, A)
    info = s.static_info(sfm.SF_STATIC_MSP)
    assert info["n_spart"] == s.info().depth + 1 and info["slack_moved"] > 0
    with pytest.raises(sfm.SparseFusionError):
        s.set_param("msp_parts", 0)
    lt = sfm.Schedule(L, None, sfm.SF_IC0_TRSV)
    with pytest.raises(sfm.SparseFusionError):
        lt.static_info(sfm.SF_STATIC_MSP)


def test_static_plans_degenerate(orc):
    """One row; a diagonal L (one wavefront); an A without rows; no unknowns
    at all (with and without rows of A): both static plans are built and
    pass the oracle's check."""
    import scipy.sparse as sp
    cases = [
        (sp.csr_matrix(np.array([[2.0]])), sp.csr_matrix(np.array([[3.0]]))),
        (sp.identity(50, format="csr") * 2.0, sp.random(30, 50, density=0.1, random_state=np.random.default_rng(1),
                                                         format="csr")),
        (sp.identity(20, format="csr") + sp.eye(20, k=-1, format="csr"), sp.csr_matrix((0, 20))),
        (sp.csr_matrix((0, 0)), sp.csr_matrix((0, 0))),
        (sp.csr_matrix((0, 0)), sp.csr_matrix((5, 0))),
    ]
    for ld, ad in cases:
        L, A = synth.from_scipy(sp.csr_matrix(ld)), synth.from_scipy(sp.csr_matrix(ad))
        s = sfm.Schedule(L, A)
        assert (s.info().depth == 0) == (L.nrows == 0)
        for plan in (sfm.SF_STATIC_MSP, sfm.SF_STATIC_WAVEFRONT):
            s_ptr, w_ptr, order = s.export_static(plan)
            assert orc.validate_static_ts(L.rowptr, L.col, A.rowptr, A.col, s_ptr, w_ptr, order) == 0, plan
            assert len(order) == L.nrows + A.nrows


@pytest.mark.filterwarnings("ignore:Sparse CSR tensor support is in beta")
def test_schedule_accepts_scipy_torch_and_tuples():
    """The same pattern given as scipy CSR, torch sparse CSR, the package's
    CSR and a (rowptr, col, ncols) tuple inspects to the same schedule; an
    unsorted row is rejected (values follow the inspected CSR order, so the
    pattern is never reordered silently)."""
    import scipy.sparse as sp
    import torch
    L, A = synth.workload("lap2d5_64")
    ref = sfm.Schedule(L, A).export()
    Ls, As = L.to_scipy(), A.to_scipy()
    Lt, At = (torch.sparse_csr_tensor(torch.as_tensor(m.indptr.astype(np.int64)),
                                      torch.as_tensor(m.indices.astype(np.int64)),
                                      torch.as_tensor(m.data), size=m.shape) for m in (Ls, As))
    for lp, ap in ((Ls, As), (Lt, At), ((L.rowptr, L.col, L.ncols), (A.rowptr, A.col, A.ncols))):
        got = sfm.Schedule(lp, ap).export()
        assert all(np.array_equal(g, r) for g, r in zip(got, ref))
    bad = sp.csr_matrix((np.ones(3), np.array([1, 0, 1]), np.array([0, 1, 3])), shape=(2, 2))
    with pytest.raises(sfm.SparseFusionError):
        sfm.Schedule(bad, None)


def test_factorisation_residency_default():
    """SpIC0 / SpILU0 schedules default to the smallest power of two (4..32)
    waves per CU that holds one wavefront's mean work items per CU (256
    CUs); SpTRSV -> SpMV schedules keep 8; set_param still overrides."""
    cases = [("lap3d27_64", sfm.SF_IC0_TRSV), ("lap3d27_64_perm", sfm.SF_IC0_TRSV),
             ("convdiff3d7_64", sfm.SF_ILU0_TRSV), ("convdiff3d7_64_perm", sfm.SF_ILU0_TRSV)]
    for name, kind in cases:
        m, _ = synth.workload(name)
        s = sfm.Schedule(m, None, kind)
        st = s.info()
        per_cu = st.n_items / st.depth / 256.0
        w = s.get_param("waves_per_cu")
        assert w in (4, 8, 16, 32) and (w == 4 or w / 2 < per_cu) and (w == 32 or w >= per_cu), (name, w, per_cu)
        s.set_param("waves_per_cu", 8)
        assert s.get_param("waves_per_cu") == 8
    got = {name: sfm.Schedule(synth.workload(name)[0], None, kind).get_param("waves_per_cu") for name, kind in cases}
    assert got == {"lap3d27_64": 4, "lap3d27_64_perm": 16, "convdiff3d7_64": 4, "convdiff3d7_64_perm": 8}
    L, A = synth.workload("lap2d5_64")
    assert sfm.Schedule(L, A).get_param("waves_per_cu") == 8


def test_structural_verdicts_match_oracle(orc):
    """sf_inspect's structural verdict on L equals the oracle's check on
    random patterns with one planted fault each (malformed CSR, an entry
    above the diagonal, a row without its diagonal, or none)."""
    import oracle_pins
    want_name = {0: None, 1: "SF_ERR_CSR", 2: "SF_ERR_NOT_LOWER", 3: "SF_ERR_ZERO_DIAG"}
    rng = np.random.default_rng(23)
    seen = set()
    for _ in range(40):
        n = int(rng.integers(1, 9))
        for name, rp, ci in oracle_pins._broken_patterns(rng, n):
            code = orc.check_lower(rp, ci)
            A = synth.from_scipy(sp.identity(n, format="csr"))
            try:
                sfm.Schedule((rp, ci, n), A).free()
                got = None
            except sfm.SparseFusionError as e:
                got = e.name
            assert got == want_name[code], (name, rp, ci)
            seen.add(code)
    assert seen == {0, 1, 2, 3}


@pytest.mark.parametrize("case,rows", [("lap3d7_20", 512), ("lap3d7_20", 64), ("lap2d9_64", 512), ("lap2d5_64", 256),
                                       ("lap3d27_10", 256), ("random", 512), ("random_rect", 128),
                                       ("tridiag", 512)])
def test_region_plans(orc, case, rows):
    """The region plan (coarsen = 3): the inspector's own check (validate)
    passes -- in-region codes, batches of one local wavefront and at most 64
    rows, external inputs listed before their first use -- and the exported
    order passes the oracle's validator with edges inside an item allowed,
    each item's rows sorted by local wavefront and every in-item edge going
    to a later one."""
    if case == "lap3d7_20":
        A = synth.laplacian_3d7(20, 20, 20, 6.0)
        L = synth.lower(A)
    elif case == "lap2d9_64":
        A = synth.laplacian_2d9(64, 64, 8.0)
        L = synth.lower(A)
    elif case == "lap2d5_64":
        A = synth.laplacian_2d5(64, 64, 4.0)
        L = synth.lower(A)
    elif case == "lap3d27_10":
        A = synth.laplacian_3d27(10, 10, 10, 26.1)
        L = synth.lower(A)
    elif case == "random":
        L, A = _random_pair(3000, 5, None, True)
    elif case == "random_rect":
        L, A = _random_pair(777, 6, 1300, True)
    else:
        A = synth.laplacian_1d(500, 2.0)
        L = synth.lower(A)
    s = sfm.Schedule(L, A, coarsen=3)
    s.set_param("region_rows", rows)
    s2 = sfm.Schedule(L, A, coarsen=3, validate=True)  # inspector's check at the default size
    assert s2.get_param("regioned") == 1
    assert s.get_param("regioned") == 1
    level, order, ip = s.export()
    loc, _ = s.export_local()
    n = L.nrows
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, ip, allow_intra=True) == 0
    item = np.repeat(np.arange(len(ip) - 1), np.diff(ip))
    pos = np.empty(len(order), np.int64)
    pos[order] = np.arange(len(order))
    for t in range(len(ip) - 1):
        seg = loc[ip[t]:ip[t + 1]]
        assert np.all(np.diff(seg.astype(int)) >= 0)
        assert np.all(order[ip[t]:ip[t + 1]] < n) or np.all(order[ip[t]:ip[t + 1]] >= n)
        if order[ip[t]] < n:
            assert ip[t + 1] - ip[t] <= rows
        else:
            assert ip[t + 1] - ip[t] <= 256  # SpMV items: 64 rows per wavefront and pass
    r = np.repeat(np.arange(n), np.diff(L.rowptr))
    off = L.col != r
    u, v = L.col[off], r[off]
    same = item[pos[u]] == item[pos[v]]
    assert np.all(loc[pos[u][same]] < loc[pos[v][same]])


def _prefix_rows_reference(L, A):
    """Rows r < min(n, m) whose A row starts with exactly L's row r
    off-diagonal columns followed by the diagonal (prefix fusion)."""
    cnt = ent = 0
    for r in range(min(L.nrows, A.nrows)):
        lc = L.col[L.rowptr[r]:L.rowptr[r + 1] - 1]
        ac = A.col[A.rowptr[r]:A.rowptr[r + 1]]
        if len(ac) >= len(lc) + 1 and np.array_equal(ac[:len(lc)], lc) and ac[len(lc)] == r:
            cnt += 1
            ent += len(lc) + 1
    return cnt, ent


@pytest.mark.parametrize("case", ["lap2d5_64", "random", "random_rect", "spd_partial"])
def test_prefix_rows(case):
    """The inspector's prefix-fusion rows match the rule written out."""
    if case == "lap2d5_64":
        L, A = synth.workload("lap2d5_64")
    elif case == "random":
        L, A = _random_pair(1000, 3)
    elif case == "random_rect":
        L, A = _random_pair(777, 6, 1300, True)
    else:
        A = synth.random_spd(3000, seed=2)
        Ls = synth.lower(A).to_scipy().tocoo()
        keep = (Ls.row == Ls.col) | (np.random.default_rng(1).random(Ls.nnz) < 0.6)
        L = synth.from_scipy(sp.csr_matrix((Ls.data[keep], (Ls.row[keep], Ls.col[keep])), shape=Ls.shape))
    s = sfm.Schedule(L, A, coarsen=1)
    want, entries = _prefix_rows_reference(L, A)
    assert s.get_param("prefix_rows") == want
    assert s.get_param("prefix_entries") == entries
    if case in ("lap2d5_64",):
        assert want == L.nrows
    if case == "spd_partial":
        assert 0 < want < L.nrows


@pytest.mark.parametrize("case,rows", [("lap3d7_16", 512), ("lap3d7_16", 64), ("lap2d9_48", 512),
                                       ("lap3d27_10", 256), ("random", 512)])
def test_backward_region_plans(orc, case, rows):
    """The backward region plan (coarsen = 3): the inspector's own check
    (validate) passes, and the exported transposed-solve order keeps every
    edge lambda_j -> lambda_i (L_ji stored, j > i) inside a region at a
    later local wavefront or across regions in claim order."""
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
        L, A = _random_pair(2000, 3)
    s = sfm.Schedule(L, A, want_backward=True, coarsen=3, validate=True)
    s.set_param("region_rows", rows)
    assert s.get_param("back_regioned") == 1
    rl, order, ip = s.export_backward()
    loc, _ = s.export_backward_local()
    n = L.nrows
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.diff(ip).max() <= min(rows, 1024)
    item = np.repeat(np.arange(len(ip) - 1), np.diff(ip))
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    for t in range(len(ip) - 1):
        assert np.all(np.diff(loc[ip[t]:ip[t + 1]].astype(int)) >= 0)
    rows_i = np.repeat(np.arange(n), np.diff(L.rowptr))
    off = L.col != rows_i
    i, j = L.col[off], rows_i[off]  # L_ji stored (j > i): lambda_j -> lambda_i
    same = item[pos[i]] == item[pos[j]]
    assert np.all(item[pos[j]][~same] < item[pos[i]][~same])
    assert np.all(loc[pos[j][same]] < loc[pos[i][same]])
