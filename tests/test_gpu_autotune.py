"""The autotuner (sf_autotune): a coordinate search over the executor's
parameters, timed on the device with the caller's data.  After tuning, the
chosen parameters are members of the candidate sets and the fused results
are still bit-identical to the oracle; a second schedule of the same pattern
takes the cached choice without timing."""
import numpy as np
import pytest

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, dev_colmajor, host

pytestmark = pytest.mark.gpu

# candidate sets of sf_autotune (defaults first)
CANDIDATES = {
    "coarsen": {0, 1, 2},
    "multi_path": {0, 1, 2},
    "rhs_block": {0, 8, 16, 32, 64},
    "spmv_delay": {-1, 1, 2, 4, 8, 16, 1 << 20},
    "rows_per_item": {64, 8, 16, 32},
    "max_item_nnz": {4096, 128, 256, 512, 1024, 2048},
    "waves_per_cu": {8, 4, 16},
    "multi_waves_per_cu": {0, 8, 16, 32},
}


def oracle_cols(orc, L, A, b):
    bb = b if b.ndim == 2 else b[:, None]
    xs = np.stack([orc.trsv_lower(L.rowptr, L.col, L.val, bb[:, c]) for c in range(bb.shape[1])], 1)
    ys = np.stack([orc.spmv(A.rowptr, A.col, A.val, xs[:, c]) for c in range(bb.shape[1])], 1)
    return (xs[:, 0], ys[:, 0]) if b.ndim == 1 else (xs, ys)


@pytest.mark.parametrize("mat,k", [("lap3d7_24", 1), ("spd_50k", 1), ("lap3d7_24", 8), ("spd_50k", 32)])
def test_autotune_keeps_results_exact_and_caches(orc, mat, k):
    import torch
    if mat == "lap3d7_24":
        A = synth.laplacian_3d7(24, 24, 24, 6.0)
    else:
        A = synth.random_spd(50_000, seed=5)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, k=k, seed=1)
    Lv, Av = dev(L.val), dev(A.val)
    B = dev(b) if k == 1 else dev_colmajor(b)
    xr, yr = oracle_cols(orc, L, A, b)
    s = sfm.Schedule(L, A)
    announce("autotune %s k=%d" % (mat, k))
    best = sfm.autotune(s, Lv, Av, B)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    assert 0.0 < best < 1e3
    assert s.get_param("tuned_from_cache") == 0
    chosen = {key: s.get_param(key) for key in CANDIDATES}
    for key, val in chosen.items():
        assert val in CANDIDATES[key], (key, val)
    announce("autotuned run %s k=%d: %s" % (mat, k, chosen))
    X, Y = sfm.trsv_spmv(s, Lv, Av, B)
    torch.cuda.synchronize()
    sfm.sync_status(s)
    assert np.array_equal(host(X), xr) and np.array_equal(host(Y), yr)
    # a new schedule of the same matrix takes the cached parameters
    s2 = sfm.Schedule(L, A)
    assert s2.get_param("fingerprint") == s.get_param("fingerprint")
    announce("autotune cache hit %s k=%d" % (mat, k))
    best2 = sfm.autotune(s2, Lv, Av, B)
    assert s2.get_param("tuned_from_cache") == 1 and best2 == best
    assert {key: s2.get_param(key) for key in CANDIDATES} == chosen
    X2, Y2 = sfm.trsv_spmv(s2, Lv, Av, B)
    torch.cuda.synchronize()
    sfm.sync_status(s2)
    assert np.array_equal(host(X2), xr) and np.array_equal(host(Y2), yr)
    s.free()
    s2.free()
