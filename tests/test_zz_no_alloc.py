"""sf_backward_noalloc, the allocation-free variant of sf_backward: the
recomputed x lives in the library's fixed device scratch instead of a
caller workspace.  Called through the C ABI and compared, bit for bit, with
sf_backward on the same inputs; two calls in a row, the second on a smaller
system, so the scratch keeps no state between calls that matters."""
import ctypes

import numpy as np
import pytest

import paper_2111_12238_amd as sfm
import synth
from gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def _lib():
    lib = sfm._lib()
    f = lib.sf_backward_noalloc
    P, I = ctypes.c_void_p, ctypes.c_int32
    f.argtypes = [P, I, P, P, P, P, P, P, P, P]
    f.restype = ctypes.c_int
    return lib


def _case(nx):
    A = synth.laplacian_3d7(nx, nx, nx, 6.0)
    L = synth.lower(A)
    return L, A


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_backward_matches_workspace_backward(dtype):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    code = 0 if dtype == "f64" else 1
    lib = _lib()
    for nx in (40, 17):  # the second call runs a smaller system on the same scratch
        L, A = _case(nx)
        n = L.nrows
        s = sfm.Schedule(L, A, want_backward=True)
        Lv, Av = dev(L.val, td), dev(A.val, td)
        b = dev(synth.vec_uniform(n, seed=1), td)
        g = dev(synth.vec_normal(A.nrows, seed=2), td)
        announce("no-alloc backward %s n=%d (forward first: makes the schedule resident)" % (dtype, n))
        X, Y = sfm.trsv_spmv(s, Lv, Av, b)
        gb_ref, gl_ref = sfm.backward(s, Lv, Av, g, B=b)  # workspace path, x recomputed
        torch.cuda.synchronize()
        gb = torch.empty(n, dtype=td, device="cuda")
        gl = torch.empty_like(Lv)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        announce("no-alloc backward call %s n=%d" % (dtype, n))
        st = lib.sf_backward_noalloc(s.handle, code, Lv.data_ptr(), Av.data_ptr(), None, b.data_ptr(),
                                     g.data_ptr(), gb.data_ptr(), gl.data_ptr(), stream)
        assert st == 0, sfm.STATUS.get(st)
        torch.cuda.synchronize()
        sfm.sync_status(s)
        assert np.array_equal(host(gb), host(gb_ref)), nx
        assert np.array_equal(host(gl), host(gl_ref)), nx
        # with the stored x no scratch is used; still the same gradients
        gb2 = torch.empty(n, dtype=td, device="cuda")
        gl2 = torch.empty_like(Lv)
        st = lib.sf_backward_noalloc(s.handle, code, Lv.data_ptr(), Av.data_ptr(), X.data_ptr(), None,
                                     g.data_ptr(), gb2.data_ptr(), gl2.data_ptr(), stream)
        assert st == 0, sfm.STATUS.get(st)
        torch.cuda.synchronize()
        assert np.array_equal(host(gb2), host(gb_ref)) and np.array_equal(host(gl2), host(gl_ref))
        s.free()


def test_noalloc_backward_needs_a_resident_schedule():
    """Before any executor call the schedule's arrays are not on the device;
    the allocation-free entry reports SF_ERR_ARG instead of allocating."""
    import torch
    lib = _lib()
    L, A = _case(8)
    s = sfm.Schedule(L, A, want_backward=True)
    Lv, Av = dev(L.val), dev(A.val)
    b, g = dev(np.ones(L.nrows)), dev(np.ones(A.nrows))
    gb, gl = torch.empty_like(b), torch.empty_like(Lv)
    announce("no-alloc backward on a schedule never executed")
    st = lib.sf_backward_noalloc(s.handle, 0, Lv.data_ptr(), Av.data_ptr(), None, b.data_ptr(), g.data_ptr(),
                                 gb.data_ptr(), gl.data_ptr(), None)
    assert st == 1  # SF_ERR_ARG
    s.free()
