"""The device probes return the machine constants the bounds use, each in a
physically plausible range for one MI355X, and leave unprobed fields at -1."""
import pytest

import paper_2111_12238_amd as sfm
from gpu_util import announce

pytestmark = pytest.mark.gpu


def test_probe_ranges():
    announce("device probe: copy, hop, gather")
    p = sfm.device_probe()
    assert 1000.0 < p["copy_GBps"] <= 8000.0, p          # under the HBM peak
    # workgroups 0 and 8 share an XCD and 0 and 1 do not when the device
    # deals workgroups to its XCDs in turn; at least one pair is measured
    hops = [p["hop_us_same_xcd"], p["hop_us_cross_xcd"]]
    assert max(hops) > 0.0, p
    assert all(h == -1.0 or 0.05 < h < 20.0 for h in hops), p
    assert 1e9 < p["gathers_per_s"] < 1e12, p
    only = sfm.device_probe(sfm.SF_PROBE_HOP)
    assert only["copy_GBps"] == -1.0 and only["gathers_per_s"] == -1.0, only
    assert max(only["hop_us_same_xcd"], only["hop_us_cross_xcd"]) > 0.0, only
