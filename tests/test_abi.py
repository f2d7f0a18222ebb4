"""The C-ABI library loads and exports every symbol include/sf.h declares;
status strings and host-only argument checks (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2111_12238_amd as sfm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sfm.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings():
    lib = sfm._lib()
    assert b"gfx950" in lib.sf_version()
    for code in range(11):
        s = lib.sf_status_str(code)
        assert s and s != b"unknown status"
    assert lib.sf_status_str(99) == b"unknown status"


def test_null_arguments_rejected_without_gpu():
    lib = sfm._lib()
    h = ctypes.c_void_p()
    assert lib.sf_inspect(None, None, None, ctypes.byref(h)) == 1  # SF_ERR_ARG
    assert lib.sf_schedule_free(None) == 0
    st = sfm.ScheduleStats()
    assert lib.sf_schedule_info(None, ctypes.byref(st)) == 1
    for fn in ("sf_exec_trsv_spmv", "sf_exec_unfused_trsv_spmv"):
        assert getattr(lib, fn)(None, 0, None, None, None, 1, 1, None, 1, None, 1, None) == 1
    assert lib.sf_exec_ic0_trsv(None, 0, None, None, None, 1, 1, None, 1, None, None) == 1
    assert lib.sf_backward(None, 0, None, None, None, None, None, None, None, None, 0, None) == 1


def test_executor_argument_checks_are_host_side():
    import synth
    L, A = synth.workload("lap2d5_16")
    s = sfm.Schedule(L, A)
    lib = sfm._lib()
    # bad dtype, bad nrhs, bad leading dimension, B aliasing X: rejected before any GPU call
    fake = ctypes.c_void_p(0x1000)
    assert lib.sf_exec_trsv_spmv(s.handle, 7, fake, fake, fake, 256, 1, ctypes.c_void_p(0x2000), 256,
                                 None, 256, None) == 1
    assert lib.sf_exec_trsv_spmv(s.handle, 0, fake, fake, fake, 256, 0, ctypes.c_void_p(0x2000), 256,
                                 None, 256, None) == 1
    assert lib.sf_exec_trsv_spmv(s.handle, 0, fake, fake, fake, 255, 1, ctypes.c_void_p(0x2000), 256,
                                 None, 256, None) == 5
    assert lib.sf_exec_trsv_spmv(s.handle, 0, fake, fake, fake, 256, 1, fake, 256, None, 256, None) == 1
    # IC0 call on a SpTRSV->SpMV schedule, FP32 IC0 on an IC0 schedule
    assert lib.sf_exec_ic0_trsv(s.handle, 0, fake, fake, None, 256, 1, None, 256, None, None) == 1
    s2 = sfm.Schedule(L, None, sfm.SF_IC0_TRSV)
    assert lib.sf_exec_ic0_trsv(s2.handle, 1, fake, fake, None, 256, 1, None, 256, None, None) == 10
    # backward without the transposed schedule
    assert lib.sf_backward(s.handle, 0, fake, fake, fake, None, fake, fake, fake, None, 0, None) == 1
    # kernel combinations 1 and 2: aliasing, missing outputs, wrong kind, rectangular A
    f2, f3 = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert lib.sf_exec_spmv_trsv(s.handle, 0, fake, fake, fake, f2, fake, None) == 1    # z aliases x
    assert lib.sf_exec_spmv_trsv(s.handle, 0, None, fake, fake, f2, f3, None) == 1      # no A values
    assert lib.sf_exec_unfused_spmv_trsv(s.handle, 0, fake, fake, fake, None, f3, None) == 1  # y needed
    assert lib.sf_exec_trsv_trsv(s.handle, 0, fake, fake, None, f3, None) == 1          # x needed
    assert lib.sf_exec_trsv_trsv(s.handle, 0, fake, fake, f2, f2, None) == 1            # x aliases z
    assert lib.sf_exec_trsv_trsv(s2.handle, 0, fake, fake, f2, f3, None) == 1           # IC0 schedule
    assert lib.sf_exec_trsv_trsv(s.handle, 3, fake, fake, f2, f3, None) == 1            # bad dtype
    Ar = synth.from_scipy(__import__("scipy.sparse", fromlist=["random"]).random(
        300, L.nrows, density=0.01, random_state=1, format="csr"))
    sr = sfm.Schedule(L, Ar)
    assert lib.sf_exec_spmv_trsv(sr.handle, 0, fake, fake, fake, f2, f3, None) == 5     # A not square
    # preconditioner apply: needs the transposed schedule, distinct vectors
    assert lib.sf_exec_ic_apply(s.handle, 0, fake, fake, f2, f3, None) == 1             # no L^T plan
    sb = sfm.Schedule(L, A, want_backward=True)
    assert lib.sf_exec_ic_apply(sb.handle, 0, fake, fake, f2, f2, None) == 1            # w aliases z
    assert lib.sf_exec_ic_apply(sb.handle, 0, fake, f2, f2, f3, None) == 1              # r aliases w
    assert lib.sf_exec_unfused_ic_apply(sb.handle, 2, fake, fake, f2, f3, None) == 1    # bad dtype


def test_params_roundtrip():
    import synth
    L, A = synth.workload("lap2d5_16")
    s = sfm.Schedule(L, A)
    assert s.get_param("multi_waves_per_cu") == 0  # by the units per level
    assert s.get_param("levelset_waves_per_cu") == 4
    for k, v in (("lanes_trsv", 8), ("lanes_spmv", 16), ("rhs_block", 32), ("waves_per_cu", 16),
                 ("multi_waves_per_cu", 32), ("levelset_waves_per_cu", 8), ("spin_limit", 12345), ("claim_streams", 4), ("rows_per_item", 32),
                 ("no_fusion", 1)):
        s.set_param(k, v)
        assert s.get_param(k) == v
    assert s.get_param("region_poll") == 64 | (2 << 16)
    assert s.get_param("precond_regions") == 1
    assert s.get_param("spmv_item_scale") == 4
    s.set_param("spmv_item_scale", 2)
    assert s.get_param("spmv_item_scale") == 2
    s.set_param("precond_regions", 0)
    assert s.get_param("precond_regions") == 0
    s.set_param("region_poll", 32 | (1 << 8) | (64 << 16))
    assert s.get_param("region_poll") == 32 | (1 << 8) | (64 << 16)
    for k, bad in (("waves_per_cu", 2), ("multi_waves_per_cu", 64), ("levelset_waves_per_cu", 3),
                   ("region_poll", 0), ("region_poll", 65), ("region_poll", 64 | (65 << 16)), ("region_poll", 1 << 24),
                   ("trace", 3), ("precond_regions", 2),
                   ("spmv_item_scale", 0), ("spmv_item_scale", 9)):
        with pytest.raises(sfm.SparseFusionError):
            s.set_param(k, bad)
    with pytest.raises(sfm.SparseFusionError):
        s.set_param("lanes_trsv", 3)
    with pytest.raises(sfm.SparseFusionError):
        s.set_param("no_such_knob", 1)
    s.set_param("coarsen", 1)  # level items (a region plan does not cut by rows_per_item)
    n_items_32 = s.info().n_items
    s.set_param("rows_per_item", 8)
    assert s.info().n_items > n_items_32


def test_device_probe_argument_checks_are_host_side():
    """Unknown probe bits and a NULL result are rejected before any device work."""
    lib = sfm._lib()
    r = sfm.ProbeResult()
    assert lib.sf_device_probe(8, ctypes.byref(r), None) == 1  # SF_ERR_ARG
    assert lib.sf_device_probe(-1, ctypes.byref(r), None) == 1  # SF_ERR_ARG
    assert lib.sf_device_probe(sfm.SF_PROBE_COPY, None, None) == 1  # SF_ERR_ARG
