"""Debug execution of the fused SpTRSV -> SpMV executor (trace mode): the
validity of a fused schedule checked on the running kernel, not only on
the order it was given -- every work item and every iteration (SpTRSV row,
SpMV row) ran exactly once, and for every edge j -> i of the joint DAG the
value of j was published before the wait of i's item for its inputs
returned (inside a coarsened item: before i's own publication).  Stamps are
the device's 100 MHz real-time counter, shared by all compute units."""
import numpy as np
import pytest

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def case_matrix(case):
    if case == "lap3d7_24":
        return synth.laplacian_3d7(24, 24, 24, 6.0)
    if case == "lap2d5_64":
        return synth.laplacian_2d5(64, 64, 4.0)
    return synth.random_spd(30_000, seed=6)


@pytest.mark.parametrize("case,coarsen", [("lap3d7_24", 1), ("lap3d7_24", 2), ("lap2d5_64", 2),
                                          ("spd_30k", 1), ("spd_30k", 2)])
def test_trace_every_iteration_once_after_its_inputs(orc, case, coarsen):
    import torch
    A = case_matrix(case)
    L = synth.lower(A)
    n, m = L.nrows, A.nrows
    b = synth.vec_uniform(n, seed=1)
    s = sfm.Schedule(L, A, coarsen=coarsen)
    s.set_param("trace", 1)
    announce("trace %s coarsen=%d" % (case, coarsen))
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    assert np.array_equal(host(X), xr)
    assert np.array_equal(host(Y), orc.spmv(A.rowptr, A.col, A.val, xr))
    items, rows = s.trace()
    level, order, item_ptr = s.export()
    n_items = len(item_ptr) - 1
    assert items.shape == (n_items, 8) and rows.shape == (n + m, 2)
    # every item ran once, every iteration was published once
    assert (items[:, 4] == 1).all(), np.unique(items[:, 4])
    assert (rows[:, 1] == 1).all(), np.unique(rows[:, 1])
    start, ready, end = (items[:, c].astype(np.int64) for c in (0, 2, 3))
    assert (start > 0).all() and (start <= ready).all() and (ready <= end).all()
    pub = rows[:, 0].astype(np.int64)
    item_of = np.repeat(np.arange(n_items), np.diff(item_ptr))[np.argsort(order, kind="stable")]
    # SpTRSV edges (j, i), j < i stored in row i of L
    ri = np.repeat(np.arange(n), np.diff(L.rowptr))
    off = L.col != ri
    i, j = ri[off], L.col[off]
    same = item_of[i] == item_of[j]
    if s.info().coarsened == 0:
        assert not same.any()  # level items hold independent rows
    cross_slack = ready[item_of[i[~same]]] - pub[j[~same]]
    assert (cross_slack >= 0).all(), int(cross_slack.min())
    assert (pub[j[same]] <= pub[i[same]]).all()
    # SpMV edges: row r of A reads x_j, iteration id n + r.  Under prefix
    # fusion (level items) a qualifying row's entries up to its diagonal are
    # folded by SpTRSV row r, which read those x_j itself: the SpMV row waits
    # for row r's publication (its partial sum) instead, and for x_j of the
    # entries past its prefix.
    rr = np.repeat(np.arange(m), np.diff(A.rowptr))
    fused = np.zeros(A.nnz, bool)
    if s.get_param("spmv_prefix") and not s.info().coarsened and not s.get_param("regioned"):
        for r in range(min(n, m)):
            lc = L.col[L.rowptr[r]:L.rowptr[r + 1] - 1]
            a0, a1 = A.rowptr[r], A.rowptr[r + 1]
            if a1 - a0 >= len(lc) + 1 and np.array_equal(A.col[a0:a0 + len(lc)], lc) and A.col[a0 + len(lc)] == r:
                fused[a0:a0 + len(lc) + 1] = True
                assert ready[item_of[n + r]] >= pub[r]
    spmv_slack = ready[item_of[n + rr[~fused]]] - pub[A.col[~fused]]
    assert (spmv_slack >= 0).all(), int(spmv_slack.min())
    print("%s coarsen=%d: %d items, %d cross-item edges (min slack %d ticks), %d in-item edges"
          % (case, coarsen, n_items, int((~same).sum()), int(cross_slack.min()) if cross_slack.size else -1,
             int(same.sum())))
    s.free()


@pytest.mark.parametrize("case,coarsen", [("lap3d7_24", 3), ("lap2d5_64", 3)])
def test_trace_region_plan(orc, case, coarsen):
    """The region plan: every region and SpMV item ran once, every row was
    published once; a row's input from another region was published before
    that region's poller had observed all its inputs, an input from its own
    region before the row's own publication."""
    test_trace_every_iteration_once_after_its_inputs(orc, case, coarsen)


@pytest.mark.parametrize("perm", [False, True])
def test_trace_ic0_every_row_once_after_its_inputs(orc, perm):
    """Fused SpIC0 -> SpTRSV in trace mode: every item ran once, every row
    was published once, and for every stored L_ij (j < i) row j -- its
    factor entries, pivot and x_j -- was published before the wait of
    row i's item for its values returned; the stamps of an item are in
    order (start <= indices loaded <= values final <= end)."""
    import torch
    a = synth.laplacian_3d27(12, 12, 12, 26.1)
    if perm:
        a = synth.permute_sym(a, synth.permutation(a.nrows, seed=3))
    Lp = synth.lower(a)
    n = Lp.nrows
    b = synth.vec_normal(n, seed=1)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    s.set_param("trace", 1)
    announce("trace ic0 27pt 12^3 perm=%s" % perm)
    Lv, X, info = sfm.ic0_trsv(s, dev(Lp.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    l, fail = orc.ic0(Lp.rowptr, Lp.col, Lp.val)
    assert np.array_equal(host(Lv), l)
    assert np.array_equal(host(X), orc.trsv_lower(Lp.rowptr, Lp.col, l, b))
    items, rows = s.trace()
    level, order, item_ptr = s.export()
    n_items = len(item_ptr) - 1
    assert (items[:, 4] == 1).all(), np.unique(items[:, 4])
    assert (rows[:n, 1] == 1).all(), np.unique(rows[:n, 1])
    start, loaded, ready, end = (items[:, c].astype(np.int64) for c in (0, 1, 2, 3))
    assert (start > 0).all() and (start <= loaded).all() and (loaded <= ready).all() and (ready <= end).all()
    pub = rows[:n, 0].astype(np.int64)
    item_of = np.repeat(np.arange(n_items), np.diff(item_ptr))[np.argsort(order, kind="stable")]
    ri = np.repeat(np.arange(n), np.diff(Lp.rowptr))
    off = Lp.col != ri
    i, j = ri[off], Lp.col[off]
    assert not (item_of[i] == item_of[j]).any()  # items hold rows of one level
    slack = ready[item_of[i]] - pub[j]
    assert (slack >= 0).all(), int(slack.min())
    print("ic0 perm=%s: %d items, %d edges, min slack %d ticks" % (perm, n_items, int(i.size), int(slack.min())))
    s.free()


@pytest.mark.parametrize("case,coarsen", [("lap3d7_24", 3), ("spd_30k", 1)])
def test_trace_items_only(orc, case, coarsen):
    """Trace level 2 stamps the items alone: every item ran exactly once
    with ordered stamps, no iteration word is written, and the results stay
    the oracle's.  On the region plan a region's stamps follow its steps:
    claimed, staged, first input stored (when it has external inputs), first
    batch published, ended."""
    import torch
    A = case_matrix(case)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, seed=2)
    s = sfm.Schedule(L, A, coarsen=coarsen)
    s.set_param("trace", 2)
    assert s.get_param("trace") == 2
    announce("trace items only %s coarsen=%d" % (case, coarsen))
    X, Y = sfm.trsv_spmv(s, dev(L.val), dev(A.val), dev(b))
    torch.cuda.synchronize()
    sfm.sync_status(s)
    xr = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    assert np.array_equal(host(X), xr)
    assert np.array_equal(host(Y), orc.spmv(A.rowptr, A.col, A.val, xr))
    items, rows = s.trace()
    assert np.all(items[:, 4] == 1), "every item runs exactly once"
    assert not rows.any(), "no iteration stamps at level 2"
    it = items.astype(np.int64)
    assert np.all(it[:, 0] <= it[:, 3]) and np.all(it[:, 0] <= it[:, 1])
    if coarsen == 3:
        assert s.get_param("regioned") == 1
        reg = it[it[:, 6] > 0]  # regions (SpMV items publish no first batch)
        assert len(reg) > 0
        assert np.all(reg[:, 0] <= reg[:, 1]) and np.all(reg[:, 1] <= reg[:, 6]) and np.all(reg[:, 6] <= reg[:, 3])
        # the first-input stamp comes from the polling wavefront, the staged
        # one from the computing wavefront just after their common barrier:
        # 1 us (100 ticks) of slack for the two wavefronts' issue order
        ext = reg[reg[:, 5] > 0]
        assert len(ext) > 0 and np.all(ext[:, 1] <= ext[:, 5] + 100)
    s.set_param("trace", 0)
