"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np


def dev(a, dtype=None):
    import torch
    if dtype is None:
        dtype = torch.float64
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def dev_colmajor(a, dtype=None):
    """(n, k) numpy array -> column-major (n, k) device tensor."""
    import torch
    if dtype is None:
        dtype = torch.float64
    t = torch.as_tensor(np.ascontiguousarray(np.asarray(a).T), dtype=dtype, device="cuda")
    return t.t()


def host(t):
    return t.detach().cpu().double().numpy()


def relerr(got, want):
    """Normwise relative error max|got - want| / max|want| (per column for 2-D)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    if want.ndim == 1:
        den = np.abs(want).max() if want.size else 1.0
        return float(np.abs(got - want).max() / (den if den > 0 else 1.0)) if want.size else 0.0
    return max(relerr(got[:, c], want[:, c]) for c in range(want.shape[1]))


def announce(msg):
    """Name the case before touching the GPU (flushed so it survives a crash)."""
    print("[case] " + msg, flush=True)
    sys.stdout.flush()
