"""Host logic of bench.py's lower bounds (no GPU): the per-matrix bounds
from a device probe pick the binding one and the fraction reached, the
gather floor applies to level-item plans only, and the critical path counts
joint wavefronts (level plan) or the longest item chain (coarsened plan)."""
import numpy as np
import pytest

import bench
import paper_2111_12238_amd as sfm
import synth

PROBE = {"copy_GBps": 4000.0, "hop_us_same_xcd": 0.4, "hop_us_cross_xcd": 0.5, "gathers_per_s": 1e11}


def _work(name, coarsen):
    L, A = synth.workload(name)
    s = sfm.Schedule(L, A)
    s.set_param("coarsen", coarsen)
    return {"s": s, "L": L, "A": A, "bytes": bench.ts_bytes(L.nrows, A.nrows, L.nnz, A.nnz)}


@pytest.mark.parametrize("coarsen", [1, 2])
def test_bounds_arithmetic(coarsen):
    d = _work("lap2d5_64", coarsen)
    st = d["s"].info()
    fused_ms = 0.05
    b = bench.bounds(d, fused_ms, PROBE)
    assert b["hbm_peak_ms"] == pytest.approx(d["bytes"] / 8e12 * 1e3, abs=1e-4)
    assert b["copy_ceiling_ms"] == pytest.approx(d["bytes"] / 4e12 * 1e3, abs=1e-4)
    gathers = d["L"].nnz - d["L"].nrows + d["A"].nnz
    if st.coarsened:
        assert b["gather_floor_ms"] is None  # in-item x comes from LDS: no floor
        assert b["critical_path_hops"] == st.chunk_chain
    else:
        assert b["gather_floor_ms"] == pytest.approx(gathers / 1e11 * 1e3, abs=1e-4)
        assert b["critical_path_hops"] == st.joint_depth
    assert b["critical_path_ms"] == pytest.approx(b["critical_path_hops"] * 0.5e-3, abs=1e-4)
    cands = {k: v for k, v in b.items() if k.endswith("_ms") and v is not None}
    top = max(cands, key=cands.get)
    assert b["binding"] == top[:-3]
    assert b["frac_of_binding"] == pytest.approx(cands[top] / fused_ms, abs=1e-3)


def test_bounds_without_probe_and_path_bound():
    d = _work("lap2d5_64", 1)
    assert bench.bounds(d, 1.0, None) is None
    assert bench.path_bound(10, 1.0, None) is None
    assert bench.path_bound(10, 1.0, dict(PROBE, hop_us_cross_xcd=-1.0, hop_us_same_xcd=-1.0)) is None
    # no cross-XCD pair placed: the same-XCD hop is charged
    assert bench.path_bound(10, 1.0, dict(PROBE, hop_us_cross_xcd=-1.0))["critical_path_ms"] == 0.004
    p = bench.path_bound(200, 0.5, PROBE)
    assert p == {"critical_path_ms": 0.1, "hops": 200, "frac_of_critical_path": 0.2}


def test_unprobed_fields_drop_out():
    """A probe field left at -1 (not measured) gives no bound of that kind."""
    d = _work("lap2d5_64", 1)
    b = bench.bounds(d, 1.0, dict(PROBE, copy_GBps=-1.0, gathers_per_s=-1.0))
    assert b["copy_ceiling_ms"] is None and b["gather_floor_ms"] is None
    assert b["binding"] in ("hbm_peak", "critical_path")
    assert np.isfinite(b["frac_of_binding"])
