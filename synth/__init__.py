"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module builds matrices and vectors only: stencil Laplacians, a random
sparse SPD matrix, symmetric permutations, lower-triangle extraction and
random right-hand sides.  It holds none of the solver's arithmetic (no
solve, product, factorisation or schedule), so both the oracle and the HIP
path can take their inputs from it without sharing any of the method.

The matrices stand in for the SuiteSparse SPD set of the paper's evaluation
(Table 1), which is not available here; they follow its shapes (SPD,
symmetric pattern, 5-33 nonzeros per row).

Recipes (all with ``numpy.random.default_rng``):
  * stencils: natural ordering (x fastest, then y, then z); 5/7-point use the
    axis neighbours, 9/27-point the whole 3^d box; off-diagonals -1, the
    diagonal a given constant on every row (boundary rows included).
  * random SPD(n, seed): row i draws 2..30 off-diagonal columns uniformly
    from the other n-1 columns; the pattern is symmetrised and deduplicated;
    each unordered pair gets one value ~ U(-1, 0) used at (i, j) and (j, i);
    the diagonal is 1 + the absolute row sum of the off-diagonals.
  * permutation(n, seed): ``default_rng(seed).permutation(n)``; the permuted
    matrix is B[k, l] = A[p[k], p[l]].
  * vectors: U(-1, 1) or N(0, 1); a block of k right-hand sides is an n x k
    column-major array.
Seeds used by the suite: matrix 0, b 1, w 2, permutation 3.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class CSR:
    """CSR matrix with int32 indices, sorted columns, float64 values."""

    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    nrows: int
    ncols: int

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.nrows, self.ncols))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def from_scipy(a) -> CSR:
    a = sp.csr_matrix(a)
    a.sum_duplicates()
    a.sort_indices()
    return CSR(np.ascontiguousarray(a.indptr, np.int32), np.ascontiguousarray(a.indices, np.int32),
               np.ascontiguousarray(a.data, np.float64), a.shape[0], a.shape[1])


def _stencil(shape, offsets, diag) -> CSR:
    """Constant-coefficient stencil on a grid in natural ordering."""
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    strides = [1]
    for s in shape[:-1]:
        strides.append(strides[-1] * s)
    offsets = sorted(offsets, key=lambda o: sum(d * st for d, st in zip(o, strides)))
    coords = np.indices(shape[::-1]).reshape(len(shape), -1)[::-1]  # coords[0] = x (fastest)
    noff = len(offsets)
    valid = np.ones((n, noff), dtype=bool)
    cols = np.empty((n, noff), dtype=np.int64)
    base = np.arange(n, dtype=np.int64)
    for k, o in enumerate(offsets):
        lin = 0
        for d, (od, sd) in enumerate(zip(o, shape)):
            c = coords[d] + od
            valid[:, k] &= (c >= 0) & (c < sd)
            lin += od * strides[d]
        cols[:, k] = base + lin
    isdiag = np.array([all(d == 0 for d in o) for o in offsets])
    vals = np.where(isdiag, float(diag), -1.0)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[valid].astype(np.int32)
    val = np.broadcast_to(vals, (n, noff))[valid].astype(np.float64)
    return CSR(rowptr.astype(np.int32), col, val, n, n)


def laplacian_2d5(nx, ny, diag=4.0) -> CSR:
    return _stencil((nx, ny), [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)], diag)


def laplacian_2d9(nx, ny, diag=8.0) -> CSR:
    offs = [(dx, dy) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return _stencil((nx, ny), offs, diag)


def laplacian_3d7(nx, ny, nz, diag=6.0) -> CSR:
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return _stencil((nx, ny, nz), offs, diag)


def laplacian_3d27(nx, ny, nz, diag=26.1) -> CSR:
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return _stencil((nx, ny, nz), offs, diag)


def laplacian_1d(n, diag=2.0) -> CSR:
    return _stencil((n,), [(0,), (-1,), (1,)], diag)


def convdiff_3d7(nx, ny, nz, diag=6.0, eps=0.4) -> CSR:
    """Nonsymmetric 3D 7-point convection-diffusion operator, natural
    ordering: off-diagonals -1 - eps toward lower coordinates (upwind) and
    -1 + eps toward higher ones, constant diagonal (input of SpILU0)."""
    a = laplacian_3d7(nx, ny, nz, diag)
    rows = np.repeat(np.arange(a.nrows), np.diff(a.rowptr))
    v = a.val.copy()
    v[a.col < rows] = -1.0 - eps
    v[a.col > rows] = -1.0 + eps
    return CSR(a.rowptr, a.col, v, a.nrows, a.ncols)


def random_nonsym(n, seed=0, lo=2, hi=12) -> CSR:
    """Random sparse nonsymmetric, diagonally dominant matrix: lo..hi
    off-diagonals per row at uniform columns (no self-loops, duplicates
    merged), values U(-1, 1), diagonal 1 + the row's absolute sum."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), counts)
    c = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    c += (c >= rows)
    m = sp.csr_matrix((rng.uniform(-1.0, 1.0, size=rows.size), (rows, c)), shape=(n, n))
    m.sum_duplicates()
    m = (m + sp.diags(np.abs(m).sum(axis=1).A1 + 1.0)).tocsr()
    m.sort_indices()
    return from_scipy(m)


def random_spd(n, seed=0, lo=2, hi=30) -> CSR:
    """Random sparse SPD matrix (recipe in the module docstring)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), counts)
    c = rng.integers(0, n - 1, size=rows.size, dtype=np.int64)
    c += (c >= rows)
    a = np.minimum(rows, c)
    b = np.maximum(rows, c)
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    v = rng.uniform(-1.0, 0.0, size=key.size)
    r = np.concatenate([a, b])
    cc = np.concatenate([b, a])
    vv = np.concatenate([v, v])
    off = sp.coo_matrix((vv, (r, cc)), shape=(n, n)).tocsr()
    diag = 1.0 + np.asarray(abs(off).sum(axis=1)).ravel()
    full = off + sp.diags(diag, format="csr")
    return from_scipy(full)


def permutation(n, seed=3) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n)


def permute_sym(a: CSR, p) -> CSR:
    """B = P A P^T, i.e. B[k, l] = A[p[k], p[l]]."""
    s = a.to_scipy()
    return from_scipy(s[p][:, p])


def lower(a: CSR) -> CSR:
    """Lower triangle including the diagonal (pattern extraction only)."""
    return from_scipy(sp.tril(a.to_scipy(), format="csr"))


def vec_uniform(n, k=1, seed=1) -> np.ndarray:
    """U(-1, 1) vector (k == 1) or n x k column-major block (shape (n, k), F order)."""
    rng = np.random.default_rng(seed)
    if k == 1:
        return rng.uniform(-1.0, 1.0, size=n)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(k, n)).T)


def vec_normal(n, k=1, seed=1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if k == 1:
        return rng.standard_normal(n)
    return np.asfortranarray(rng.standard_normal(size=(k, n)).T)


def random_lower(n, density, seed=0, int_values=False) -> CSR:
    """Random lower-triangular matrix with a dominant diagonal (test inputs)."""
    rng = np.random.default_rng(seed)
    m = sp.random(n, n, density=density, random_state=rng, format="csr")
    m = sp.tril(m, k=-1, format="csr")
    if int_values:
        m.data = rng.integers(-3, 4, size=m.nnz).astype(np.float64)
        m.data[m.data == 0] = 1.0
        d = rng.choice([1.0, 2.0, 4.0], size=n)
    else:
        m.data = rng.uniform(-1.0, 1.0, size=m.nnz)
        d = 1.0 + np.asarray(abs(m).sum(axis=1)).ravel()
    return from_scipy(m + sp.diags(d, format="csr"))


def int_vector(n, seed=5, lo=-8, hi=8) -> np.ndarray:
    """Integer-valued float64 vector in [lo, hi] (manufactured solutions)."""
    return np.random.default_rng(seed).integers(lo, hi + 1, size=n).astype(np.float64)


# Workload catalogue: name -> (builder, description).  Sizes follow the
# configurations the suite measures.
def workload(name: str):
    """Return (L, A) or (lower(A), A) for a named workload."""
    if name == "lap2d5_64":
        a = laplacian_2d5(64, 64, 4.0)
    elif name == "lap2d5_16":
        a = laplacian_2d5(16, 16, 4.0)
    elif name == "lap3d7_128":
        a = laplacian_3d7(128, 128, 128, 6.0)
    elif name == "lap3d7_96":
        a = laplacian_3d7(96, 96, 96, 6.0)
    elif name == "randspd_1m":
        a = random_spd(1_000_000, seed=0)
    elif name == "lap3d27_64":
        a = laplacian_3d27(64, 64, 64, 26.1)
    elif name == "lap3d27_64_perm":
        a0 = laplacian_3d27(64, 64, 64, 26.1)
        a = permute_sym(a0, permutation(a0.nrows, seed=3))
    elif name == "lap2d9_2048":
        a = laplacian_2d9(2048, 2048, 8.0)
    elif name in ("convdiff3d7_64", "convdiff3d7_64_perm", "randnonsym_1m"):
        # SpILU0 inputs: the whole nonsymmetric matrix is the pattern
        if name == "randnonsym_1m":
            a = random_nonsym(1_000_000, seed=0)
        else:
            a = convdiff_3d7(64, 64, 64, 6.0, 0.4)
            if name.endswith("_perm"):
                a = permute_sym(a, permutation(a.nrows, seed=3))
        return a, a
    else:
        raise KeyError(name)
    return lower(a), a
