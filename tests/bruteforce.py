"""Dense brute-force references for small inputs (n <= 64).

They pin the oracle from outside: each is written from the dense linear
algebra definition (LAPACK through scipy, or an explicit O(n^3) loop in a
different loop order than the oracle's), never by calling the oracle.
"""
import numpy as np
import scipy.linalg as sl


def solve_lower(ld, b):
    return sl.solve_triangular(ld, b, lower=True)


def solve_upper_t(ld, c):
    return sl.solve_triangular(ld.T, c, lower=False)


def ic0_right_looking(ad, mask):
    """Zero fill-in incomplete Cholesky by the right-looking (outer-product)
    recurrence on a dense copy: column k is scaled, then every later entry
    (i, j) that is inside the lower pattern is updated.  Returns (L, first
    failing column or -1)."""
    n = ad.shape[0]
    a = np.tril(ad).astype(np.float64).copy()
    m = np.tril(mask).astype(bool)
    fail = -1
    for k in range(n):
        if not (a[k, k] > 0) and fail < 0:
            fail = k
        a[k, k] = np.sqrt(a[k, k]) if a[k, k] > 0 else np.nan
        for i in range(k + 1, n):
            if m[i, k]:
                a[i, k] = a[i, k] / a[k, k]
        for j in range(k + 1, n):
            if not m[j, k]:
                continue
            for i in range(j, n):
                if m[i, k] and m[i, j]:
                    a[i, j] -= a[i, k] * a[j, k]
    return np.where(m, a, 0.0), fail


def levels_longest_path(ld):
    """Longest path from any source in the DAG j -> i for L_ij != 0 (j < i),
    by dynamic programming over a dense adjacency with the Bellman recurrence
    iterated to a fixed point (independent of row order)."""
    n = ld.shape[0]
    adj = (ld != 0) & ~np.eye(n, dtype=bool)
    lv = np.zeros(n, dtype=np.int64)
    for _ in range(n + 1):
        cand = np.where(adj, lv[None, :] + 1, 0).max(axis=1) if n else lv
        new = np.maximum(lv, cand)
        if np.array_equal(new, lv):
            break
        lv = new
    return lv


def dense_gradients(ld, ad, b, w):
    """loss = w^T A L^{-1} b.  Returns (x, grad_b, grad_L dense masked)."""
    x = solve_lower(ld, b)
    lam = solve_upper_t(ld, ad.T @ w)
    gl = -np.outer(lam, x) * (ld != 0)
    return x, lam, gl


def _merges(seqs):
    """Every interleaving of the sequences that keeps each one's order."""
    seqs = [list(s) for s in seqs if len(s)]
    if not seqs:
        yield []
        return
    for k, s in enumerate(seqs):
        rest = seqs[:k] + [s[1:]] + seqs[k + 1:]
        for tail in _merges(rest):
            yield [s[0]] + tail


def static_schedule_runs(n_vertices, preds, s_ptr, w_ptr, order):
    """Simulate a two-level static schedule: the s-partitions in sequence,
    the w-partitions of one s-partition in every possible interleaving.
    True iff every vertex runs exactly once, after all of its predecessors,
    in every execution."""
    import itertools
    if sorted(order) != list(range(n_vertices)):
        return False
    per_s = []
    for b in range(len(s_ptr) - 1):
        ws = [order[w_ptr[w]:w_ptr[w + 1]] for w in range(s_ptr[b], s_ptr[b + 1])]
        per_s.append(list(_merges(ws)))
    for choice in itertools.product(*per_s):
        done = set()
        for part in choice:
            for v in part:
                if any(u not in done for u in preds[v]):
                    return False
                done.add(v)
    return True


def item_schedule_runs(n_vertices, preds, order, item_ptr, together):
    """Simulate an item schedule: items run one after another; the
    iterations of one item start together and read their inputs as the item
    starts, except that ``together(u, v)`` names the pairs (u, v) one item
    runs back to back on the same lanes (v then sees u's result if u is
    listed first).  True iff every vertex runs exactly once and every
    predecessor's result exists when it is read."""
    if sorted(order) != list(range(n_vertices)):
        return False
    if item_ptr[0] != 0 or item_ptr[-1] != len(order):
        return False
    if any(item_ptr[t + 1] <= item_ptr[t] for t in range(len(item_ptr) - 1)):
        return False
    done = set()
    for t in range(len(item_ptr) - 1):
        members = order[item_ptr[t]:item_ptr[t + 1]]
        for k, v in enumerate(members):
            earlier_here = set(members[:k])
            for u in preds[v]:
                if u in done:
                    continue
                if u in earlier_here and together(u, v):
                    continue
                return False
        done.update(members)
    return True


def csr_status(rp, ci, nrows, ncols, lower):
    """Structural verdict of a CSR pattern through scipy's own format
    checks: 1 malformed (row pointers, column range, order or duplicates),
    2 an entry above the diagonal, 3 a row without its diagonal, 0 valid
    (2 and 3 only when ``lower``)."""
    import scipy.sparse as sp
    rp = np.asarray(rp, np.int64)
    ci = np.asarray(ci, np.int64)
    if len(rp) != nrows + 1 or rp[0] != 0 or np.any(np.diff(rp) < 0) or rp[-1] > len(ci):
        return 1
    ci = ci[:rp[-1]]
    try:
        a = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(nrows, ncols))
        a.check_format(full_check=True)
    except ValueError:
        return 1
    if not a.has_canonical_format:  # sorted columns without duplicates in every row
        return 1
    if lower:
        if sp.triu(a, 1).nnz:
            return 2
        if np.any(a.diagonal() == 0):
            return 3
    return 0
