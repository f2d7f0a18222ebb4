"""GPU parity of the fused SpILU0 -> SpTRSV executor (Table 2, combination
6) and its level-set baseline against the oracle: L, U and y bit for bit in
FP64, zero pivots reported at the oracle's row."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def run_ilu(s, a, x, unfused=False, check=True):
    import torch
    LU, Y, info = sfm.ilu0_trsv(s, dev(a.val), None if x is None else dev(x), unfused=unfused, check_info=check)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    return host(LU), (None if Y is None else host(Y)), int(info.item())


def oracle_ilu(orc, a, x):
    lu, fail = orc.ilu0(a.rowptr, a.col, a.val)
    y = orc.trsv_unit_lower(a.rowptr, a.col, lu, x)
    return lu, y, fail


CASES = {
    "convdiff_12": lambda: synth.convdiff_3d7(12, 12, 12),
    "convdiff_perm": lambda: synth.permute_sym(synth.convdiff_3d7(10, 9, 8), synth.permutation(720, seed=3)),
    "random_nonsym": lambda: synth.random_nonsym(5000, seed=2),
    "lap27_8": lambda: synth.laplacian_3d27(8, 8, 8, 26.1),
    "tridiag": lambda: synth.from_scipy(sp.diags([np.full(299, -1.5), np.full(300, 4.0), np.full(299, -0.5)],
                                                 [-1, 0, 1], format="csr")),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_ilu0_trsv_bit_identical(orc, name):
    announce("ilu0 fused " + name)
    a = CASES[name]()
    x = synth.vec_normal(a.nrows, seed=1)
    lr, yr, fail = oracle_ilu(orc, a, x)
    assert fail == -1
    s = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV)
    for unfused in (False, True):
        lu, y, info = run_ilu(s, a, x, unfused=unfused)
        assert info == -1
        assert np.array_equal(lu, lr) and np.array_equal(y, yr), unfused


def test_ilu0_small_items_and_factor_only(orc):
    announce("ilu0 small items / factor only")
    a = synth.random_nonsym(3000, seed=7, lo=1, hi=6)
    x = synth.vec_normal(a.nrows, seed=2)
    lr, yr, _ = oracle_ilu(orc, a, x)
    s = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV, rows_per_item=1, lanes_per_row=32)
    lu, y, _ = run_ilu(s, a, x)
    assert np.array_equal(lu, lr) and np.array_equal(y, yr)
    lu, y, info = run_ilu(s, a, None)
    assert y is None and info == -1 and np.array_equal(lu, lr)


def test_ilu0_zero_pivot_reports_first_row(orc):
    """Rows 120 and 300 get a zero pivot; d_info holds the oracle's first
    failing row and the launch completes (fused and level-set)."""
    announce("ilu0 zero pivot")
    n = 400
    m = sp.diags([np.full(n - 1, -1.0), np.full(n, 4.0), np.full(n - 1, -2.0)], [-1, 0, 1], format="csr")
    # make u_120 and u_300 exactly zero: a_ii = l_i,i-1 * u_i-1,i (the one subtracted term)
    for r in (120, 300):
        lu, _ = orc.ilu0(m.indptr, m.indices, m.data)
        full = sp.csr_matrix((lu, m.indices, m.indptr)).tolil()
        m = m.tolil()
        m[r, r] = full[r, r - 1] * full[r - 1, r]
        m = m.tocsr()
    a = synth.from_scipy(m)
    _, _, fail = oracle_ilu(orc, a, np.ones(n))
    assert fail == 120
    s = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV)
    for unfused in (False, True):
        _, _, info = run_ilu(s, a, np.ones(n), unfused=unfused, check=False)
        assert info == fail
    with pytest.raises(sfm.SparseFusionError) as e:
        run_ilu(s, a, np.ones(n))
    assert e.value.row == 120


def test_ilu0_rows_longer_than_lanes_rejected():
    announce("ilu0 long rows rejected (host check)")
    a = synth.convdiff_3d7(6, 6, 6)
    s = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV, lanes_per_row=4)
    with pytest.raises(sfm.SparseFusionError) as e:
        run_ilu(s, a, np.ones(a.nrows))
    assert e.value.name == "SF_ERR_UNSUPPORTED"


@pytest.mark.parametrize("name", ["convdiff3d7_64", "convdiff3d7_64_perm"])
def test_ilu0_full_size(orc, name):
    announce("ilu0 full size " + name)
    a, _ = synth.workload(name)
    x = synth.vec_normal(a.nrows, seed=1)
    lr, yr, fail = oracle_ilu(orc, a, x)
    s = sfm.Schedule(a, None, sfm.SF_ILU0_TRSV)
    lu, y, info = run_ilu(s, a, x)
    assert fail == info == -1
    assert np.array_equal(lu, lr) and np.array_equal(y, yr)
