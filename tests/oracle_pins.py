"""Pins of the oracle against facts fixed by the mathematics or the paper.

Each ``pin_*`` takes an oracle object (``oracle.Oracle``) and raises
AssertionError when the oracle disagrees.  The same pins run against the
real oracle (test_oracle_pins.py) and against copies of it with planted
mistakes (test_oracle_mutants.py), which must each fail at least one pin.
"""
import os

import numpy as np
import scipy.sparse as sp

import bruteforce as bf
import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

U64 = 2.0 ** -53


def _csr(d):
    return synth.from_scipy(sp.csr_matrix(d))


def _bidiag(n):
    d = np.diag(np.full(n, 2.0)) + np.diag(np.full(n - 1, -1.0), -1)
    return _csr(d)


# ---------------------------------------------------------------- SpTRSV ----
def pin_trsv_bidiag_closed_form(orc):
    """L = bidiag(2 on the diagonal, -1 below): (L^{-1})_ij = 2^{-(i-j)-1}
    for i >= j, and b = 1 gives x_i = 1 - 2^{-(i+1)} (0-based).  Every value
    is a dyadic rational, exact in FP64, so the check is bit-exact."""
    n = 50
    L = _bidiag(n)
    x = orc.trsv_lower(L.rowptr, L.col, L.val, np.ones(n))
    want = 1.0 - 2.0 ** -(np.arange(n) + 1.0)
    assert np.array_equal(x, want), "bidiagonal ones-RHS"
    for j in (0, 7, 31):
        e = np.zeros(n)
        e[j] = 1.0
        col = orc.trsv_lower(L.rowptr, L.col, L.val, e)
        i = np.arange(n)
        wantc = np.where(i >= j, 2.0 ** (-(i - j) - 1.0), 0.0)
        assert np.array_equal(col, wantc), "bidiagonal inverse column %d" % j


def pin_trsv_round_trip_integer(orc):
    """Integer L (integer diagonal from {1,2,4}) and integer x_true: b = L x_true
    is exact, each partial sum of forward substitution is an integer, and the
    division by L_ii is exact, so x must equal x_true bit for bit."""
    for seed, n, dens in ((0, 60, 0.1), (1, 500, 0.02), (2, 3000, 0.003)):
        L = synth.random_lower(n, dens, seed=seed, int_values=True)
        xt = synth.int_vector(n, seed=seed + 10)
        b = L.to_scipy() @ xt
        x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
        assert np.array_equal(x, xt), "integer round trip n=%d" % n


def pin_trsv_dense_bruteforce(orc):
    """Random sparse lower L (n <= 64) against LAPACK dtrtrs, normwise."""
    for seed in range(4):
        L = synth.random_lower(48, 0.2, seed=seed)
        b = synth.vec_uniform(48, seed=seed)
        x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
        ref = bf.solve_lower(L.dense(), b)
        assert np.abs(x - ref).max() <= 1e-13 * np.abs(ref).max()


def pin_trsv_backward_error_bound(orc):
    """Forward substitution is componentwise backward stable in any order:
    |b - L x| <= gamma_m |L| |x| with m the largest row length (Higham,
    Accuracy and Stability of Numerical Algorithms, Ch. 8)."""
    L, _ = synth.workload("lap2d5_64")
    a = synth.random_spd(20000, seed=7)
    for Lm in (L, synth.lower(a)):
        n = Lm.nrows
        b = synth.vec_uniform(n, seed=3)
        x = orc.trsv_lower(Lm.rowptr, Lm.col, Lm.val, b)
        s = Lm.to_scipy()
        m = int(np.diff(Lm.rowptr).max())
        gam = m * U64 / (1 - m * U64)
        r = np.abs(b - s @ x)
        bound = gam * (abs(s) @ np.abs(x))
        assert np.all(r <= bound * 1.0000001 + 1e-300), "backward error bound"


# ------------------------------------------------------------------ SpMV ----
def pin_spmv(orc):
    """Integer SpMV is exact in any order; a float SpMV agrees with scipy to
    the inner-product bound gamma_m |A||x|."""
    _, A = synth.workload("lap2d5_64")
    xi = synth.int_vector(A.ncols, seed=2)
    y = orc.spmv(A.rowptr, A.col, A.val, xi)
    assert np.array_equal(y, A.to_scipy() @ xi)
    a = synth.random_spd(3000, seed=1)
    x = synth.vec_uniform(3000, seed=4)
    y = orc.spmv(a.rowptr, a.col, a.val, x)
    s = a.to_scipy()
    m = int(np.diff(a.rowptr).max())
    bound = 2 * m * U64 * (abs(s) @ np.abs(x))
    assert np.all(np.abs(y - s @ x) <= bound)
    # rectangular with an empty row: y = 0 there
    r = sp.csr_matrix(np.array([[1.0, 0, 2.0], [0, 0, 0], [0, 3.0, 0]]))
    c = synth.from_scipy(r)
    y = orc.spmv(c.rowptr, c.col, c.val, np.array([1.0, 2.0, 3.0]))
    assert np.array_equal(y, [7.0, 0.0, 6.0])


def pin_transpose_products(orc):
    """c = A^T g against the dense transpose; the transpose round-trips."""
    a = synth.random_spd(40, seed=5)
    sa = sp.csr_matrix(a.dense()[:30, :])  # rectangular 30 x 40
    A = synth.from_scipy(sa)
    g = synth.vec_normal(30, seed=2)
    c = orc.spmv_t(A.rowptr, A.col, A.val, g, 40)
    ref = sa.toarray().T @ g
    assert np.abs(c - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    trp, tci, perm = orc.transpose(A.rowptr, A.col, 40)
    t = sp.csr_matrix((A.val[perm], tci, trp), shape=(40, 30)).toarray()
    assert np.array_equal(t, sa.toarray().T)


def pin_trsv_upper_t(orc):
    """Upper solve L^T lam = c against LAPACK, and the 1D Laplacian inverse:
    with T = tridiag(-1, 2, -1) = L L^T (L its exact Cholesky factor),
    (T^{-1})_ij = min(i, j) (n + 1 - max(i, j)) / (n + 1), 1-based."""
    for seed in range(3):
        L = synth.random_lower(40, 0.2, seed=seed)
        c = synth.vec_uniform(40, seed=seed + 1)
        lam = orc.trsv_upper_t(L.rowptr, L.col, L.val, c)
        ref = bf.solve_upper_t(L.dense(), c)
        assert np.abs(lam - ref).max() <= 1e-13 * np.abs(ref).max()
    n = 40
    T = synth.laplacian_1d(n, 2.0)
    Lt = synth.lower(T)
    lval, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
    assert fail == -1
    i1 = np.arange(1, n + 1)
    for k in (1, 17, 40):
        e = np.zeros(n)
        e[k - 1] = 1.0
        z = orc.trsv_lower(Lt.rowptr, Lt.col, lval, e)
        col = orc.trsv_upper_t(Lt.rowptr, Lt.col, lval, z)
        want = np.minimum(i1, k) * (n + 1 - np.maximum(i1, k)) / (n + 1)
        assert np.abs(col - want).max() <= 1e-12, "T^-1 column %d" % k


# ------------------------------------------------------------------ SpIC0 ----
def pin_ic0_tridiagonal_closed_form(orc):
    """IC0 of tridiag(-1, 2, -1) has no dropped fill, so it is the exact
    Cholesky factor: L_ii = sqrt((i+1)/i), L_{i+1,i} = -sqrt(i/(i+1)),
    1-based."""
    n = 64
    Lt = synth.lower(synth.laplacian_1d(n, 2.0))
    lval, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
    assert fail == -1
    ld = sp.csr_matrix((lval, Lt.col, Lt.rowptr), shape=(n, n)).toarray()
    i = np.arange(1, n + 1, dtype=np.float64)
    # a few ulps of rounding accumulate along the recurrence
    assert np.abs(np.diag(ld) - np.sqrt((i + 1) / i)).max() <= 16 * U64
    sub = np.diag(ld, -1)
    assert np.abs(sub - (-np.sqrt(i[:-1] / i[1:]))).max() <= 16 * U64


def pin_ic0_no_fill_equals_cholesky(orc):
    """When the Cholesky factor has no fill outside lower(A) (dense SPD, and
    block-diagonal with dense blocks), IC0 equals LAPACK dpotrf."""
    rng = np.random.default_rng(11)
    m = rng.standard_normal((24, 24))
    ad = m @ m.T + 24 * np.eye(24)
    blocks = [ad[:10, :10], ad[10:, 10:]]
    bd = np.zeros((24, 24))
    bd[:10, :10] = blocks[0]
    bd[10:, 10:] = blocks[1]
    for d in (ad, bd):
        Lt = _csr(np.tril(d))
        lval, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
        assert fail == -1
        ld = sp.csr_matrix((lval, Lt.col, Lt.rowptr), shape=d.shape).toarray()
        ref = np.linalg.cholesky(d)
        assert np.abs(ld - ref).max() <= 1e-13 * np.abs(ref).max()


def pin_ic0_dense_masked_bruteforce(orc):
    """Sparse SPD patterns (n <= 64): the up-looking oracle against a
    right-looking dense masked recurrence; the two agree in exact
    arithmetic."""
    for seed in range(3):
        a = synth.random_spd(50, seed=seed, lo=2, hi=5)
        Lt = synth.lower(a)
        lval, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
        ad = a.dense()
        ref, rfail = bf.ic0_right_looking(ad, ad != 0)
        assert fail == rfail == -1
        ld = sp.csr_matrix((lval, Lt.col, Lt.rowptr), shape=ad.shape).toarray()
        assert np.abs(ld - ref).max() <= 1e-13 * np.abs(ref).max()


def pin_ic0_invariants(orc):
    """On the 27-point stencil (12^3, diagonal 26.1), natural and permuted:
    (L L^T)_ij = A_ij on the pattern within the rounding bound
    gamma_{m+1} (|L||L^T|)_ij, and every pivot is positive."""
    a0 = synth.laplacian_3d27(12, 12, 12, 26.1)
    for a in (a0, synth.permute_sym(a0, synth.permutation(a0.nrows, seed=3))):
        Lt = synth.lower(a)
        lval, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
        assert fail == -1
        ls = sp.csr_matrix((lval, Lt.col, Lt.rowptr), shape=(a.nrows, a.nrows))
        prod = (ls @ ls.T).tocsr()
        absprod = (abs(ls) @ abs(ls).T).tocsr()
        m = int(np.diff(Lt.rowptr).max()) + 1
        gam = m * U64 / (1 - m * U64)
        lt = Lt.to_scipy().tocoo()
        err = np.abs(np.asarray(prod[lt.row, lt.col]).ravel() - lt.data)
        bound = gam * np.asarray(absprod[lt.row, lt.col]).ravel()
        assert np.all(err <= bound), "L L^T = A on the pattern"
        assert np.all(lval[Lt.col == np.repeat(np.arange(a.nrows), np.diff(Lt.rowptr))] > 0)


def pin_ic0_breakdown_row(orc):
    """A non-positive pivot is reported at the first failing row, matching the
    dense recurrence."""
    d = np.array([[1.0, -2.0, 0.0, 0.0], [-2.0, 1.0, 0.0, 0.0],
                  [0.0, 0.0, 1.0, 0.5], [0.0, 0.0, 0.5, 1.0]])
    Lt = _csr(np.tril(d))
    _, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
    _, rfail = bf.ic0_right_looking(d, d != 0)
    assert fail == rfail == 1
    d3 = np.array([[1.0, -2.0, 0.0, 0.0], [-2.0, 1.0, 0.0, 0.0],
                   [0.0, 0.0, 1.0, -2.0], [0.0, 0.0, -2.0, 1.0]])  # rows 1 and 3 fail
    Lt = _csr(np.tril(d3))
    _, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
    _, rfail = bf.ic0_right_looking(d3, d3 != 0)
    assert fail == rfail == 1
    d2 = np.array([[4.0, 1.0, 0.0], [1.0, 4.0, 3.9], [0.0, 3.9, 3.0]])
    Lt = _csr(np.tril(d2))
    _, fail = orc.ic0(Lt.rowptr, Lt.col, Lt.val)
    _, rfail = bf.ic0_right_looking(d2, d2 != 0)
    assert fail == rfail == 2


# ----------------------------------------------------------------- levels ----
def pin_levels_stencil_closed_forms(orc):
    """Natural-order stencils: level(x, y) = x + y (5-point), x + 2y
    (9-point), level(x, y, z) = x + y + z (7-point), x + 2y + 4z (27-point).
    Depths 2m-1, 3m-2, 3m-2, 7m-6 on an m-sided grid."""
    cases = [
        (synth.laplacian_2d5(9, 7), (9, 7), lambda x, y: x + y),
        (synth.laplacian_2d9(9, 7), (9, 7), lambda x, y: x + 2 * y),
        (synth.laplacian_3d7(7, 6, 5), (7, 6, 5), lambda x, y, z: x + y + z),
        (synth.laplacian_3d27(7, 6, 5), (7, 6, 5), lambda x, y, z: x + 2 * y + 4 * z),
        (synth.laplacian_2d5(64, 64), (64, 64), lambda x, y: x + y),
    ]
    for a, shape, f in cases:
        L = synth.lower(a)
        lv, depth = orc.levels(L.rowptr, L.col)
        coords = np.indices(shape[::-1]).reshape(len(shape), -1)[::-1]
        want = f(*coords)
        assert np.array_equal(lv, want)
        assert depth == want.max() + 1
    for mside, (builder, k) in ((16, (synth.laplacian_2d5, 2)), (16, (synth.laplacian_2d9, 3))):
        L = synth.lower(builder(mside, mside))
        assert orc.levels(L.rowptr, L.col)[1] == k * mside - (k - 1)


def pin_levels_bruteforce(orc):
    """Levels equal the longest-path lengths found by a dense fixed-point
    iteration; reverse levels equal those of the transposed DAG."""
    for seed in range(4):
        L = synth.random_lower(60, 0.08, seed=seed)
        ld = L.dense()
        lv, depth = orc.levels(L.rowptr, L.col)
        ref = bf.levels_longest_path(ld)
        assert np.array_equal(lv, ref) and depth == ref.max() + 1
        rl, rdepth = orc.reverse_levels(L.rowptr, L.col)
        # transposed DAG: reverse the index order so it is lower again
        p = np.arange(59, -1, -1)
        rref = bf.levels_longest_path(ld.T[np.ix_(p, p)])[p]
        assert np.array_equal(rl, rref) and rdepth == rref.max() + 1


def pin_joint_order(orc):
    """SpMV row r is ready one wavefront after the last x_j it reads
    (F = pattern of A); the canonical order is sorted by (joint level,
    SpTRSV before SpMV, row), checked with numpy's lexsort."""
    L, A = synth.workload("lap2d5_16")
    lv, _ = orc.levels(L.rowptr, L.col)
    ready = orc.spmv_ready(A.rowptr, A.col, lv)
    ad = A.dense() != 0
    want = np.array([lv[np.nonzero(ad[r])[0]].max() + 1 for r in range(A.nrows)])
    assert np.array_equal(ready, want)
    order = orc.joint_order_ts(lv, ready)
    n, m = L.nrows, A.nrows
    keys_lv = np.concatenate([lv, ready])
    kind = np.concatenate([np.zeros(n, int), np.ones(m, int)])
    row = np.concatenate([np.arange(n), np.arange(m)])
    ref = np.lexsort((row, kind, keys_lv))
    assert np.array_equal(order, ref)
    # an empty SpMV row has joint level 0
    e = synth.from_scipy(sp.csr_matrix(np.array([[0.0, 0.0], [1.0, 1.0]])))
    r = orc.spmv_ready(e.rowptr, e.col, np.array([0, 1], np.int32))
    assert np.array_equal(r, [0, 2])


def pin_validator(orc):
    """The schedule check accepts the canonical per-level items and rejects
    each mutation: two dependent rows swapped, a row dropped, a row
    duplicated, a dependent pair placed in one item."""
    L, A = synth.workload("lap2d5_16")
    n, m = L.nrows, A.nrows
    lv, _ = orc.levels(L.rowptr, L.col)
    ready = orc.spmv_ready(A.rowptr, A.col, lv)
    order = orc.joint_order_ts(lv, ready)
    key = np.concatenate([lv, ready])[order] * 2 + (order >= n)
    cuts = np.nonzero(np.diff(key))[0] + 1
    item_ptr = np.concatenate([[0], cuts, [n + m]]).astype(np.int32)
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, item_ptr) == 0
    # swap TRSV row 0 with its dependent row 1 (both singleton positions)
    bad = order.copy()
    i0, i1 = np.nonzero(order == 0)[0][0], np.nonzero(order == 1)[0][0]
    bad[i0], bad[i1] = bad[i1], bad[i0]
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, bad, item_ptr) != 0
    dup = order.copy()
    dup[-1] = dup[0]
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, dup, item_ptr) != 0
    short = item_ptr.copy()
    short[-1] -= 1
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, short) != 0
    # every SpTRSV row in one item, then one item per SpMV row: only L edges
    # fall inside an item
    trsv_first = np.concatenate([order[order < n], order[order >= n]]).astype(np.int32)
    ptr2 = np.concatenate([[0], np.arange(n, n + m + 1)]).astype(np.int32)
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, trsv_first, ptr2) != 0
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, trsv_first, ptr2, allow_intra=True) == 0
    merged = np.array([0, n + m], np.int32)  # one item holding everything
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, merged) != 0
    assert orc.validate_ts(L.rowptr, L.col, A.rowptr, A.col, order, merged, allow_intra=True) == 0


def _broken_patterns(rng, n):
    """A valid lower-triangular pattern (random, diagonal last in each row)
    and copies of it with one planted structural fault each."""
    d = np.tril((rng.random((n, n)) < 0.3).astype(float), -1) + np.eye(n)
    a = sp.csr_matrix(d)
    a.sort_indices()
    rp, ci = a.indptr.astype(np.int32), a.indices.astype(np.int32)
    out = [("valid", rp, ci)]
    rows = [r for r in range(n) if rp[r + 1] - rp[r] >= 2]
    if rows:
        r = int(rng.choice(rows))
        c = ci.copy()
        c[rp[r]], c[rp[r] + 1] = c[rp[r] + 1], c[rp[r]]
        out.append(("unsorted", rp, c))
        c = ci.copy()
        c[rp[r] + 1] = c[rp[r]]
        out.append(("duplicate", rp, c))
    c = ci.copy()
    c[int(rng.integers(0, len(c)))] = n + int(rng.integers(0, 3))
    out.append(("column_range", rp, c))
    c = ci.copy()
    c[int(rng.integers(0, len(c)))] = -1 - int(rng.integers(0, 3))
    out.append(("negative_column", rp, c))
    if n >= 2:
        p = rp.copy()
        k = int(rng.integers(1, n + 1))
        p[k] = p[k - 1] - 1  # row k - 1 ends before it starts; the rows before it are untouched
        out.append(("rowptr_decreasing", p, ci))
    p = rp.copy()
    p[0] = 1
    out.append(("rowptr_start", p, ci))
    # an entry above the diagonal: row r gets column n - 1 appended after its diagonal
    r = int(rng.integers(0, n - 1)) if n >= 2 else None
    if r is not None:
        dd = d.copy()
        dd[r, n - 1] = 1.0
        b = sp.csr_matrix(dd)
        b.sort_indices()
        out.append(("upper", b.indptr.astype(np.int32), b.indices.astype(np.int32)))
    # a row without its diagonal
    dd = d.copy()
    dd[int(rng.integers(0, n)), :] = 0.0
    dd[:, :] = np.where(np.eye(n, dtype=bool) & (dd.sum(1, keepdims=True) == 0), 0.0, dd)
    b = sp.csr_matrix(dd)
    b.sort_indices()
    out.append(("no_diagonal", b.indptr.astype(np.int32), b.indices.astype(np.int32)))
    return out


def pin_csr_checks_against_scipy(orc):
    """The structural checks agree with scipy's CSR format checks
    (row pointers, column range, sorted columns without duplicates) and with
    the triangular and diagonal tests of the lower-triangular case, on
    random patterns with one planted fault each: malformed CSR is 1, an
    entry above the diagonal 2, a row without its diagonal 3, valid 0."""
    rng = np.random.default_rng(11)
    seen = set()
    for _ in range(60):
        n = int(rng.integers(1, 9))
        for name, rp, ci in _broken_patterns(rng, n):
            want_l = bf.csr_status(rp, ci, n, n, lower=True)
            want_g = bf.csr_status(rp, ci, n, n, lower=False)
            assert orc.check_lower(rp, ci) == want_l, (name, rp, ci)
            assert orc.check_csr(rp, ci, n) == want_g, (name, rp, ci)
            seen.add((name, want_l))
            if name == "valid":
                # the same pattern read as a general matrix with fewer columns
                nc = int(ci.max()) if len(ci) else 0
                assert orc.check_csr(rp, ci, nc) == bf.csr_status(rp, ci, n, nc, lower=False)
    names = {k for k, _ in seen}
    assert {"valid", "unsorted", "duplicate", "column_range", "upper", "no_diagonal"} <= names
    assert {v for _, v in seen} == {0, 1, 2, 3}


def _level_items_it(orc, L):
    """Canonical factor -> solve schedule: per level, each row's factor
    iteration directly followed by its solve iteration, one item per level."""
    n = L.nrows
    lv, depth = orc.levels(L.rowptr, L.col)
    rows = np.argsort(lv, kind="stable")
    order = np.empty(2 * n, np.int32)
    order[0::2] = rows
    order[1::2] = rows + n
    counts = np.bincount(lv, minlength=depth)
    item_ptr = np.concatenate([[0], 2 * np.cumsum(counts)]).astype(np.int32)
    return order, item_ptr


def pin_factor_solve_validator(orc):
    """The factorisation -> SpTRSV schedule check (F = I) agrees with a
    simulation of item-by-item execution on 400 tiny random DAGs and
    schedules, accepts the canonical per-level schedule of a stencil and
    rejects its mutations: dependent rows in one item, a solve row ahead of
    its factor row, a dependent row moved ahead of its input, a dropped
    iteration."""
    rng = np.random.default_rng(5)
    n_valid = 0
    for _ in range(400):
        n = int(rng.integers(1, 6))
        ld = np.tril((rng.random((n, n)) < 0.4).astype(float), -1) + np.eye(n)
        L = synth.from_scipy(sp.csr_matrix(ld))
        preds = [[j for j in range(i) if ld[i, j]] for i in range(n)]
        preds += [[j + n for j in range(i) if ld[i, j]] + [i] for i in range(n)]
        if rng.random() < 0.5:
            order, item_ptr = _level_items_it(orc, L)
            order, item_ptr = list(order), list(item_ptr)
            if rng.random() < 0.5:  # split or merge some items
                cuts = sorted(set(int(c) for c in rng.integers(1, 2 * n, int(rng.integers(0, 3)))) |
                              set(item_ptr[1:-1]))
                if rng.random() < 0.5 and cuts:
                    cuts.remove(cuts[int(rng.integers(0, len(cuts)))])
                item_ptr = [0] + cuts + [2 * n]
        else:
            order = [int(v) for v in rng.permutation(2 * n)]
            k = int(rng.integers(0, 2 * n))
            item_ptr = [0] + sorted(set(int(c) for c in rng.integers(1, 2 * n, k))) + [2 * n]
        want = bf.item_schedule_runs(2 * n, preds, order, item_ptr, lambda u, v: u < n and v == u + n)
        got = orc.validate_factor_solve(L.rowptr, L.col, np.array(order, np.int32), np.array(item_ptr, np.int32))
        assert (got == 0) == want, (got, want, order, item_ptr, ld)
        n_valid += int(want)
    assert 40 <= n_valid <= 360
    a = synth.laplacian_3d27(4, 3, 3, 26.1)
    L = synth.lower(a)
    n = L.nrows
    order, ip = _level_items_it(orc, L)
    assert orc.validate_factor_solve(L.rowptr, L.col, order, ip) == 0
    assert orc.validate_factor_solve(L.rowptr, L.col, order, np.array([0, 2 * n], np.int32)) != 0
    sw = order.copy()
    sw[0], sw[1] = sw[1], sw[0]                      # solve row before its factor row
    assert orc.validate_factor_solve(L.rowptr, L.col, sw, ip) != 0
    mv = order.copy()
    k = int(np.nonzero(mv == n - 1)[0][0])           # the last row's factor iteration ...
    mv[[0, k]] = mv[[k, 0]]                          # ... swapped into the first item
    assert orc.validate_factor_solve(L.rowptr, L.col, mv, ip) != 0
    dup = order.copy()
    dup[-1] = dup[0]
    assert orc.validate_factor_solve(L.rowptr, L.col, dup, ip) != 0


def _random_static_case(rng):
    """A tiny joint SpTRSV -> SpMV DAG and a two-level schedule of it: half
    the time cut from a random topological order (often valid), otherwise
    a random assignment (mostly invalid)."""
    n, m = int(rng.integers(2, 6)), int(rng.integers(0, 4))
    ld = np.tril((rng.random((n, n)) < 0.45).astype(float), -1) + np.eye(n)
    ad = (rng.random((m, n)) < 0.4).astype(float)
    L, A = synth.from_scipy(sp.csr_matrix(ld)), synth.from_scipy(sp.csr_matrix(ad, shape=(m, n)))
    preds = [[j for j in range(i) if ld[i, j]] for i in range(n)] + [[j for j in range(n) if ad[r, j]]
                                                                      for r in range(m)]
    N = n + m
    if rng.random() < 0.5:
        # a topological order: every SpTRSV row in row order, each SpMV row
        # after its last input, then random cuts
        order = list(range(n))
        for r in range(m):
            at = max([order.index(j) + 1 for j in preds[n + r]] + [int(rng.integers(0, len(order) + 1))])
            order.insert(at, n + r)
    else:
        order = [int(v) for v in rng.permutation(N)]
    nb = int(rng.integers(1, 4))
    scuts = sorted(int(c) for c in rng.integers(0, N + 1, nb - 1))
    s_bounds = [0] + scuts + [N]
    s_ptr, w_ptr, ords = [0], [0], []
    for b in range(nb):
        chunk = order[s_bounds[b]:s_bounds[b + 1]]
        nw = int(rng.integers(1, 4))
        owner = rng.integers(0, nw, len(chunk))
        for w in range(nw):
            part = [v for v, o in zip(chunk, owner) if o == w]
            ords += part
            w_ptr.append(len(ords))
        s_ptr.append(s_ptr[-1] + nw)
    return L, A, preds, N, np.array(s_ptr, np.int32), np.array(w_ptr, np.int32), np.array(ords, np.int32)


def pin_static_validator_bruteforce(orc):
    """The static-schedule check agrees with a simulation of every
    interleaving of the w-partitions of each s-partition (s-partitions in
    sequence) on 300 tiny random DAGs and schedules; dropped and duplicated
    vertices are rejected."""
    rng = np.random.default_rng(7)
    n_valid = 0
    for _ in range(300):
        L, A, preds, N, s_ptr, w_ptr, order = _random_static_case(rng)
        want = bf.static_schedule_runs(N, preds, list(s_ptr), list(w_ptr), list(order))
        got = orc.validate_static_ts(L.rowptr, L.col, A.rowptr, A.col, s_ptr, w_ptr, order)
        assert (got == 0) == want, (got, want, s_ptr, w_ptr, order)
        n_valid += int(want)
        if N >= 2:
            dup = order.copy()
            dup[-1] = dup[0]
            assert orc.validate_static_ts(L.rowptr, L.col, A.rowptr, A.col, s_ptr, w_ptr, dup) != 0
    assert 30 <= n_valid <= 270  # both verdicts are exercised


def pin_reuse_ratio(orc):
    """Reuse ratios from the paper's formulas (Sec. 2.2; Table 2,
    combinations 4 and 5) against the hand-computed values stored in
    tests/golden/reuse_ratio.txt; combination 4 is < 1 and 5 is >= 1."""
    rows = _golden("reuse_ratio.txt")
    for r in rows:
        kind, n, nnz_l, m, nnz_a, want = r[0], int(r[1]), int(r[2]), int(r[3]), int(r[4]), float(r[5])
        got = orc.reuse_ts(n, nnz_l, m, nnz_a) if kind == "ts" else orc.reuse_it(n, nnz_l)
        assert abs(got - want) <= 1e-15 * want
        assert (got < 1.0) if kind == "ts" else (got >= 1.0)


# -------------------------------------------------------------- gradients ----
def pin_gradients_fd_and_dense(orc):
    """loss = <w, A L^{-1} b> on the 2D 5-point 16x16 Laplacian: the adjoint
    against central finite differences (h = 1e-6, FP64) for every entry of
    b and every stored value of L, and against the dense formulas
    grad_b = L^{-T} A^T w, grad_L = -(grad_b x^T) masked to the pattern."""
    L, A = synth.workload("lap2d5_16")
    n = L.nrows
    b = synth.vec_uniform(n, seed=1)
    w = synth.vec_normal(n, seed=2)
    x = orc.trsv_lower(L.rowptr, L.col, L.val, b)
    gb, gl = orc.backward(L.rowptr, L.col, L.val, A.rowptr, A.col, A.val, x, w)
    xd, gbd, gld = bf.dense_gradients(L.dense(), A.dense(), b, w)
    assert np.abs(gb - gbd).max() <= 1e-12 * np.abs(gbd).max()
    rows = np.repeat(np.arange(n), np.diff(L.rowptr))
    assert np.abs(gl - gld[rows, L.col]).max() <= 1e-12 * np.abs(gld).max()

    def loss(lv, bv):
        xx = orc.trsv_lower(L.rowptr, L.col, lv, bv)
        return float(w @ orc.spmv(A.rowptr, A.col, A.val, xx))

    h = 1e-6
    fd_b = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd_b[i] = (loss(L.val, b + e) - loss(L.val, b - e)) / (2 * h)
    fd_l = np.empty(L.nnz)
    for p in range(L.nnz):
        e = np.zeros(L.nnz)
        e[p] = h
        fd_l[p] = (loss(L.val + e, b) - loss(L.val - e, b)) / (2 * h)
    tol_b = 1e-7 * max(1.0, np.abs(gb).max())
    tol_l = 1e-7 * max(1.0, np.abs(gl).max())
    assert np.abs(gb - fd_b).max() <= tol_b
    assert np.abs(gl - fd_l).max() <= tol_l


def _golden(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                out.append(ln.split())
    return out


# ---------------------------------------------------------------- SpILU0 ----
def _ilu_factors(orc, a):
    lu, fail = orc.ilu0(a.rowptr, a.col, a.val)
    d = sp.csr_matrix((lu, a.col, a.rowptr), shape=(a.nrows, a.nrows)).toarray()
    n = a.nrows
    return np.tril(d, -1) + np.eye(n), np.triu(d), fail


def pin_ilu0_tridiagonal_is_lu(orc):
    """A tridiagonal matrix has no fill, so ILU0 is its LU factorisation;
    diagonal dominance makes LAPACK's partial pivoting pick no row swap, so
    scipy.linalg.lu must return the same factors (nonsymmetric values)."""
    import scipy.linalg as la
    n = 40
    rng = np.random.default_rng(4)
    d = (np.diag(rng.uniform(4, 5, n)) + np.diag(rng.uniform(-1, 0, n - 1), -1)
         + np.diag(rng.uniform(-2, 1, n - 1), 1))
    a = _csr(d)
    Lm, Um, fail = _ilu_factors(orc, a)
    P, Lr, Ur = la.lu(d)
    assert fail == -1 and np.array_equal(P, np.eye(n)), "no pivoting expected"
    assert np.abs(Lm - Lr).max() <= 8 * U64 and np.abs(Um - Ur).max() <= 8 * U64 * np.abs(Ur).max()


def pin_ilu0_product_matches_on_pattern(orc):
    """The defining property: (L U)_ij = A_ij for every stored (i, j), with L
    unit lower and U upper on the pattern of A (nonsymmetric patterns and
    values, fill positions outside the pattern not constrained)."""
    for seed, n in ((1, 60), (2, 200)):
        rng = np.random.default_rng(seed)
        m = sp.random(n, n, density=6.0 / n, random_state=rng, format="csr")
        m.data = rng.uniform(-1, 1, m.nnz)
        m = (m + sp.diags(np.abs(m).sum(1).A1 + 1.0)).tocsr()
        m.sort_indices()
        a = synth.from_scipy(m)
        Lm, Um, fail = _ilu_factors(orc, a)
        assert fail == -1
        prod = Lm @ Um
        mask = m.toarray() != 0
        mask[np.diag_indices(n)] = True
        err = np.abs(prod - m.toarray())[mask].max()
        assert err <= 64 * U64 * np.abs(m.toarray()).max(), ("LU on pattern", seed, err)
        assert np.all(Lm[~mask & (np.tril(np.ones((n, n)), -1) > 0)] == 0)
        assert np.all(Um[~mask & (np.triu(np.ones((n, n))) > 0)] == 0)


def pin_ilu0_symmetric_matches_ic0(orc):
    """On a symmetric positive definite matrix with symmetric pattern, ILU0
    and IC0 are the same factorisation up to scaling: with C the IC0 factor,
    L = C diag(C)^{-1} and U = diag(C) C^T (the pinned IC0 above)."""
    a = synth.laplacian_3d27(5, 4, 4, 26.1)
    lower = synth.lower(a)
    c, fail_c = orc.ic0(lower.rowptr, lower.col, lower.val)
    Lm, Um, fail = _ilu_factors(orc, a)
    assert fail == -1 and fail_c == -1
    C = sp.csr_matrix((c, lower.col, lower.rowptr), shape=(a.nrows, a.nrows)).toarray()
    dc = np.diag(C)
    assert np.abs(Lm - C / dc[None, :]).max() <= 32 * U64
    assert np.abs(Um - dc[:, None] * C.T).max() <= 64 * U64 * np.abs(Um).max()


def pin_ilu0_zero_pivot_row(orc):
    """A zero pivot (u_11 = 0 after elimination) is reported at its row;
    the first of two failing rows is the one returned."""
    d = np.array([[2.0, 1.0, 0.0, 0.0], [4.0, 2.0, 1.0, 0.0], [0.0, 1.0, 3.0, 1.0], [0.0, 0.0, 3.0, 1.0]])
    # row 1: u_11 = 2 - (4/2) * 1 = 0
    _, _, fail = _ilu_factors(orc, _csr(d))
    assert fail == 1
    # rows 2 and 4 have no stored diagonal: the first of them is reported
    _, _, fail2 = _ilu_factors(orc, _csr(np.diag([1.0, 1.0, 0.0, 1.0, 0.0])))
    assert fail2 == 2


def pin_trsv_unit_lower(orc):
    """Unit-lower solve: integer L below the diagonal (any stored diagonal or
    upper entries are ignored) and integer y give integer b exactly; the
    solve must return y bit for bit."""
    rng = np.random.default_rng(5)
    n = 300
    m = sp.random(n, n, density=0.02, random_state=rng, format="csr")
    m.data = rng.integers(-2, 3, m.nnz).astype(np.float64)
    m = (m + sp.diags(np.full(n, 7.0))).tocsr()
    m.sort_indices()
    a = synth.from_scipy(m)
    low = sp.tril(m, -1).toarray() + np.eye(n)
    y = rng.integers(-5, 6, n).astype(np.float64)
    b = low @ y
    assert np.array_equal(orc.trsv_unit_lower(a.rowptr, a.col, a.val, b), y)


# ------------------------------------------------------------ refinement ----
def _refine(orc, L, A, b, ncorr, l32=None):
    return orc.refine(L.rowptr, L.col, L.val, A.rowptr, A.col, A.val, b, ncorr, l32=l32)


def pin_refine_diagonal_is_one_fp32_division(orc):
    """Diagonal L: the FP32 substitution reduces to fl32(fl32(b_i) / L32_ii)
    (numpy's float32 division, correctly rounded); the FP64 residual of that
    is then corrected, and y = A x is the plain FP64 product."""
    rng = np.random.default_rng(31)
    n = 400
    d = rng.uniform(0.5, 3.0, n)
    L = _csr(np.diag(d))
    A = L
    b = rng.uniform(-1, 1, n)
    x, y, rel, st = _refine(orc, L, A, b, 0)
    want = b.astype(np.float32) / d.astype(np.float32)
    assert np.array_equal(st[:, 0], want) and np.array_equal(x, want.astype(np.float64)), "x0 of diagonal L"
    x1, y1, rel1, st1 = _refine(orc, L, A, b, 1)
    r = b - d * want.astype(np.float64)  # exact in FP64: one product, one difference per row
    d1 = r.astype(np.float32) / d.astype(np.float32)
    assert np.array_equal(st1[:, 1], d1), "first correction of diagonal L"
    assert np.array_equal(x1, want.astype(np.float64) + d1.astype(np.float64)), "x1 of diagonal L"
    assert np.array_equal(y1, d * x1), "y = A x, diagonal A"


def pin_refine_integer_system_is_exact(orc):
    """Integer L (diagonals from {1,2,4}, entries exactly representable in
    FP32) and integer x_true with b = L x_true: every FP32 partial sum is a
    small integer and every division exact, so x0 = x_true, each residual is
    0, every correction is 0, and x = x_true bit for bit; y = A x_true."""
    for seed, n, dens in ((0, 80, 0.1), (1, 700, 0.015)):
        L = synth.random_lower(n, dens, seed=seed, int_values=True)
        xt = synth.int_vector(n, seed=seed + 10)
        b = L.to_scipy() @ xt
        A = synth.from_scipy(L.to_scipy() + L.to_scipy().T)
        for nc in (0, 2):
            x, y, rel, st = _refine(orc, L, A, b, nc)
            assert np.array_equal(x, xt), "integer refinement n=%d ncorr=%d" % (n, nc)
            assert np.array_equal(y, A.to_scipy() @ xt), "integer y n=%d" % n
            assert rel == 0.0 and (st[:, 1:] == 0).all(), "zero residual and corrections"


def pin_refine_converges_to_fp64_solution(orc):
    """The refinement's fixed point is the FP64 solution: on SPD-derived L
    (random SPD, 2D 9-point, 3D 7-point) the FP32-only x0 is ~1e-7 away from
    LAPACK's FP64 triangular solve, each correction cuts the error by about
    that factor, and two corrections are within 1e-13; the reported relative
    residual equals max|b - L x| / max|b| recomputed with scipy (its own
    summation) to within rounding; y is within 1e-14 of scipy's A @ x."""
    from scipy.linalg import solve_triangular
    cases = (synth.random_spd(3000, seed=2), synth.laplacian_2d9(40, 40, 8.0), synth.laplacian_3d7(12, 12, 12, 6.0))
    for A in cases:
        L = synth.lower(A)
        n = L.nrows
        b = synth.vec_uniform(n, seed=1)
        Ls = L.to_scipy()
        xr = solve_triangular(Ls.toarray(), b, lower=True) if n <= 3000 else None
        errs = []
        for nc in (0, 1, 2):
            x, y, rel, st = _refine(orc, L, A, b, nc)
            errs.append(np.abs(x - xr).max() / np.abs(xr).max())
            res = np.abs(b - Ls @ x).max() / np.abs(b).max()
            assert abs(rel - res) <= 1e-15 * max(1.0, np.abs(xr).max()), (nc, rel, res)
            yy = A.to_scipy() @ x
            assert np.abs(y - yy).max() <= 1e-14 * np.abs(yy).max(), "y = A x"
        assert 1e-9 < errs[0] < 1e-5, errs
        assert errs[1] < errs[0] * 1e-4 and errs[2] <= 1e-13, errs


def pin_refine_fp32_substitution_backward_error(orc):
    """The FP32 stage is a substitution with FP32 arithmetic: its result
    satisfies the componentwise backward-error bound of forward
    substitution (any summation order), |c - L32 v| <= gamma_{m+1} |L32||v|
    with u = 2^-24, m the longest row (Higham, Ch. 8), evaluated in FP64."""
    A = synth.random_spd(2000, seed=9)
    L = synth.lower(A)
    b = synth.vec_uniform(L.nrows, seed=4)
    x, y, rel, st = _refine(orc, L, A, b, 0)
    v = st[:, 0].astype(np.float64)
    L32 = sp.csr_matrix((L.val.astype(np.float32).astype(np.float64), L.col, L.rowptr), shape=(L.nrows, L.nrows))
    c = b.astype(np.float32).astype(np.float64)
    m = int(np.diff(L.rowptr).max())
    u = 2.0 ** -24
    gam = (m + 1) * u / (1 - (m + 1) * u)
    lhs = np.abs(c - L32 @ v)
    rhs = gam * (abs(L32) @ np.abs(v)) + u * np.abs(c)
    assert (lhs <= rhs).all(), float((lhs - rhs).max())
    # and it is not an FP64 solve: x0 differs from the FP64 solution
    assert not np.array_equal(x, np.linalg.solve(L.to_scipy().toarray(), b))


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
