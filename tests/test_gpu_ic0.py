"""GPU parity of the fused SpIC0 -> SpTRSV executor (and its level-set
baseline) against the oracle: factor values and solution within 1e-12
normwise relative, breakdown row identical."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host, relerr

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def run_ic0(s, Lp, b, unfused=False, check=True):
    import torch
    Av = dev(Lp.val)
    Lv, X, info = sfm.ic0_trsv(s, Av, None if b is None else dev(b), unfused=unfused, check_info=check)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    return host(Lv), (None if X is None else host(X)), int(info.item())


def oracle_it(orc, Lp, b):
    l, fail = orc.ic0(Lp.rowptr, Lp.col, Lp.val)
    x = orc.trsv_lower(Lp.rowptr, Lp.col, l, b)
    return l, x, fail


@pytest.mark.parametrize("perm", [False, True])
def test_27pt_12cube(orc, perm):
    announce("ic0 fused 27pt 12^3 perm=%s" % perm)
    a = synth.laplacian_3d27(12, 12, 12, 26.1)
    if perm:
        a = synth.permute_sym(a, synth.permutation(a.nrows, seed=3))
    Lp = synth.lower(a)
    b = synth.vec_normal(a.nrows, seed=1)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    l, x, info = run_ic0(s, Lp, b)
    lr, xr, fail = oracle_it(orc, Lp, b)
    assert info == fail == -1
    assert relerr(l, lr) <= TOL64 and relerr(x, xr) <= TOL64
    lu, xu, infou = run_ic0(s, Lp, b, unfused=True)
    assert infou == -1
    assert relerr(lu, lr) <= TOL64 and relerr(xu, xr) <= TOL64
    # every term of the recurrences, rounded once, in the oracle's order
    nd = int(np.sum(l != lr)), int(np.sum(x != xr))
    print("27pt perm=%s values differing from the oracle: L %d x %d" % (perm, nd[0], nd[1]))
    assert np.array_equal(l, lr) and np.array_equal(x, xr)
    assert np.array_equal(lu, lr) and np.array_equal(xu, xr)


@pytest.mark.parametrize("lanes,name", [(4, "lap2d5_64"), (8, "lap2d9_64")])
def test_small_lane_groups_bit_identical(orc, lanes, name):
    """Rows of at most 4 and 8 entries on groups of 4 and 8 lanes (several
    groups share one 16-lane DPP row): L and x bit-identical to the oracle."""
    announce("ic0 fused %s lanes=%d" % (name, lanes))
    a = synth.laplacian_2d5(64, 64, 4.0) if name == "lap2d5_64" else synth.laplacian_2d9(64, 64, 8.0)
    Lp = synth.lower(a)
    assert np.diff(Lp.rowptr).max() <= lanes
    b = synth.vec_normal(Lp.nrows, seed=4)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV, lanes_per_row=lanes)
    assert s.get_param("lanes_trsv") == lanes
    lr, xr, fail = oracle_it(orc, Lp, b)
    assert fail == -1
    for unfused in (False, True):
        l, x, info = run_ic0(s, Lp, b, unfused=unfused)
        assert info == -1 and np.array_equal(l, lr) and np.array_equal(x, xr), unfused


def test_tridiagonal_closed_form():
    """IC0 of tridiag(-1, 2, -1) is its exact Cholesky factor:
    L_ii = sqrt((i+1)/i), L_{i+1,i} = -sqrt(i/(i+1)) (1-based)."""
    announce("ic0 fused tridiagonal closed form")
    n = 1000
    Lp = synth.lower(synth.laplacian_1d(n, 2.0))
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    l, x, info = run_ic0(s, Lp, np.ones(n))
    assert info == -1
    ld = sp.csr_matrix((l, Lp.col, Lp.rowptr), shape=(n, n))
    i = np.arange(1, n + 1, dtype=np.float64)
    assert np.abs(ld.diagonal() - np.sqrt((i + 1) / i)).max() <= 64 * 2.0 ** -53
    assert np.abs(ld.diagonal(-1) + np.sqrt(i[:-1] / i[1:])).max() <= 64 * 2.0 ** -53


@pytest.mark.parametrize("lanes,lo,hi", [(16, 1, 3), (32, 2, 6), (64, 2, 6)])
def test_random_spd_patterns(orc, lanes, lo, hi):
    announce("ic0 fused random spd lanes=%d" % lanes)
    a = synth.random_spd(5000, seed=9, lo=lo, hi=hi)
    Lp = synth.lower(a)
    assert np.diff(Lp.rowptr).max() - 1 <= lanes  # one lane per stored entry of a row
    b = synth.vec_normal(a.nrows, seed=2)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV, lanes_per_row=lanes, rows_per_item=17)
    l, x, info = run_ic0(s, Lp, b)
    lr, xr, fail = oracle_it(orc, Lp, b)
    assert info == fail == -1
    assert relerr(l, lr) <= TOL64 and relerr(x, xr) <= TOL64


def test_rows_longer_than_lanes_rejected():
    announce("ic0 long rows rejected (host check)")
    a = synth.random_spd(5000, seed=9, lo=2, hi=6)
    Lp = synth.lower(a)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV, lanes_per_row=16)
    with pytest.raises(sfm.SparseFusionError) as e:
        run_ic0(s, Lp, np.ones(a.nrows))
    assert e.value.name == "SF_ERR_UNSUPPORTED"


def test_breakdown_reports_first_row(orc):
    """A non-positive pivot: d_info holds the smallest failing row (the
    oracle's), and the launch still completes."""
    announce("ic0 fused breakdown")
    n = 400
    d = sp.diags([np.full(n - 1, -1.0), np.full(n, 2.0), np.full(n - 1, -1.0)], [-1, 0, 1]).tolil()
    d[150, 150] = 0.4
    d[300, 300] = -1.0
    Lp = synth.lower(synth.from_scipy(d.tocsr()))
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    _, _, fail = oracle_it(orc, Lp, np.ones(n))
    assert fail == 150
    for unfused in (False, True):
        _, _, info = run_ic0(s, Lp, np.ones(n), unfused=unfused, check=False)
        assert info == fail
    with pytest.raises(sfm.SparseFusionError) as e:
        run_ic0(s, Lp, np.ones(n))
    assert e.value.row == 150


def test_factor_only(orc):
    announce("ic0 fused factor only")
    a = synth.laplacian_3d27(10, 9, 8, 26.1)
    Lp = synth.lower(a)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    l, x, info = run_ic0(s, Lp, None)
    lr, _, _ = oracle_it(orc, Lp, np.zeros(a.nrows))
    assert x is None and info == -1 and relerr(l, lr) <= TOL64


@pytest.mark.parametrize("name", ["lap3d27_64", "lap3d27_64_perm"])
def test_full_size(orc, name):
    announce("ic0 fused full size " + name)
    Lp, _ = synth.workload(name)
    b = synth.vec_normal(Lp.nrows, seed=1)
    s = sfm.Schedule(Lp, None, sfm.SF_IC0_TRSV)
    l, x, info = run_ic0(s, Lp, b)
    lr, xr, fail = oracle_it(orc, Lp, b)
    print("%s: L err %.2e x err %.2e depth %d" % (name, relerr(l, lr), relerr(x, xr), s.info().depth))
    assert info == fail == -1
    assert relerr(l, lr) <= TOL64 and relerr(x, xr) <= TOL64
