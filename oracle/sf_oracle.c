/*
 * Sequential FP64 reference ("oracle") for the fused sparse executor.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table
 * or helper with the HIP path.
 *
 * Every routine is the plain definition of the operation it computes,
 * written out in row order with ascending column order inside a row.  It is
 * compiled with -ffp-contract=off so no multiply-add is fused.
 *
 * Sources (Cheshmi, Strout, Mehri Dehnavi, "Composing Loop-carried
 * Dependence with Other Loops", arXiv 2111.12238):
 *   - SpTRSV solves L x = b and SpMV computes y = A x (Sec. 1, the running
 *     example of Fig. 2).
 *   - The SpTRSV dependence DAG is the pattern of L: a stored L_ij is an
 *     edge from iteration j to iteration i (Sec. 2.2, "Dependency DAGs").
 *   - F_ij != 0 means iteration j of the first loop must precede iteration
 *     i of the second loop (Sec. 2.2, "Dependency Matrix F"; Sec. 3.1).
 *   - Wavefront (level-set) parallelism over the DAG (Sec. 1; "fused
 *     wavefront" baseline, Sec. 4 setup).
 *   - A fused partitioning runs its s-partitions in sequence and the
 *     independent w-partitions of one s-partition in parallel, each
 *     w-partition's iterations in order (Sec. 3.1, output of MSP).
 *   - SpIC0 is zero fill-in incomplete Cholesky, L L^T ~= A (Table 2,
 *     combinations 5 and 7).  The paper gives no recurrence; the one used
 *     here is the textbook up-looking row form: the unique lower-triangular
 *     L with pattern(L) = pattern(lower(A)) and (L L^T)_ij = A_ij on that
 *     pattern.
 *   - Reuse ratio = common accesses / max(accesses of each kernel)
 *     (Sec. 2.2, "Reuse Ratio"; Table 2 last column).
 *   - SpILU0 is zero fill-in incomplete LU, L U ~= A (Table 2, combinations
 *     3 and 6).  The paper gives no recurrence; the one used here is
 *     row-wise Gaussian elimination restricted to the pattern of A (the IKJ
 *     variant): the unique unit-lower L and upper U on pattern(A) with
 *     (L U)_ij = A_ij on that pattern.
 *   - Adjoint of y = A L^{-1} b (not in the paper): with g = dloss/dy,
 *     lambda = L^{-T} (A^T g), grad_b = lambda, grad_L = -lambda x^T
 *     restricted to the pattern of L.
 *
 *   - Mixed-precision refinement of x = L^{-1} b (not in the paper): FP32
 *     substitutions with FP32 accumulation, FP64 residuals r = b - L x, the
 *     FP32 correction solved from the rounded residual and added in FP64,
 *     then y = A x in FP64.  In each FP32 substitution the off-diagonal
 *     products are summed first (ascending column, from 0) and the sum is
 *     subtracted from the rounded right-hand side: every row's sums then
 *     need no value of the row's own chain (see orc_refine).
 *
 * Parity pins: every function here is pinned by tests/test_oracle_*.py
 * against closed forms, dense brute force (numpy / LAPACK) and invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status codes of the oracle's structural check (its own numbering). */
#define ORC_OK 0
#define ORC_BAD_CSR 1       /* rowptr not monotone, column out of range, unsorted or duplicate */
#define ORC_NOT_LOWER 2     /* an entry with column > row */
#define ORC_NO_DIAG 3       /* a row of L without its diagonal entry */

/* Structural check of a lower-triangular CSR matrix with sorted columns. */
int orc_check_lower(int n, const int32_t* rp, const int32_t* ci) {
  if (rp[0] != 0) return ORC_BAD_CSR;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return ORC_BAD_CSR;
    int has_diag = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j < 0 || j >= n) return ORC_BAD_CSR;
      if (p > rp[i] && ci[p - 1] >= j) return ORC_BAD_CSR;
      if (j > i) return ORC_NOT_LOWER;
      if (j == i) has_diag = 1;
    }
    if (!has_diag) return ORC_NO_DIAG;
  }
  return ORC_OK;
}

/* Structural check of a general m x ncols CSR matrix with sorted columns. */
int orc_check_csr(int m, int ncols, const int32_t* rp, const int32_t* ci) {
  if (rp[0] != 0) return ORC_BAD_CSR;
  for (int i = 0; i < m; ++i) {
    if (rp[i + 1] < rp[i]) return ORC_BAD_CSR;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j < 0 || j >= ncols) return ORC_BAD_CSR;
      if (p > rp[i] && ci[p - 1] >= j) return ORC_BAD_CSR;
    }
  }
  return ORC_OK;
}

/* SpTRSV, forward substitution: x_i = (b_i - sum_{j<i} L_ij x_j) / L_ii,
 * rows in order 0..n-1, off-diagonal terms subtracted in ascending column
 * order. */
void orc_trsv_lower(int n, const int32_t* rp, const int32_t* ci, const double* v,
                    const double* b, double* x) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    double d = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j < i) s -= v[p] * x[j];
      else if (j == i) d = v[p];
    }
    x[i] = s / d;
  }
}

/* SpMV: y_i = sum_p A[p] x[col[p]], ascending p. */
void orc_spmv(int m, const int32_t* rp, const int32_t* ci, const double* v,
              const double* x, double* y) {
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) s += v[p] * x[ci[p]];
    y[i] = s;
  }
}

/* Explicit transpose of an m x ncols CSR matrix into CSR of the ncols x m
 * transpose (rows of the result ascending in source row).  perm[q] is the
 * position in the source arrays of transposed entry q. */
void orc_transpose(int m, int ncols, const int32_t* rp, const int32_t* ci,
                   int32_t* trp, int32_t* tci, int32_t* perm) {
  for (int j = 0; j <= ncols; ++j) trp[j] = 0;
  for (int p = 0; p < rp[m]; ++p) trp[ci[p] + 1] += 1;
  for (int j = 0; j < ncols; ++j) trp[j + 1] += trp[j];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncols > 0 ? ncols : 1));
  for (int j = 0; j < ncols; ++j) fill[j] = trp[j];
  for (int i = 0; i < m; ++i)
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int q = fill[ci[p]]++;
      tci[q] = i;
      perm[q] = p;
    }
  free(fill);
}

/* Transposed SpMV, by its definition c_j = sum_r A_rj g_r with r ascending,
 * evaluated over an explicit transpose. */
void orc_spmv_t(int m, int ncols, const int32_t* rp, const int32_t* ci, const double* v,
                const double* g, double* c) {
  int32_t* trp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ncols + 1));
  int32_t* tci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(rp[m] > 0 ? rp[m] : 1));
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(rp[m] > 0 ? rp[m] : 1));
  orc_transpose(m, ncols, rp, ci, trp, tci, perm);
  for (int j = 0; j < ncols; ++j) {
    double s = 0.0;
    for (int q = trp[j]; q < trp[j + 1]; ++q) s += v[perm[q]] * g[tci[q]];
    c[j] = s;
  }
  free(trp); free(tci); free(perm);
}

/* Upper solve with the transpose of a lower-triangular L: L^T lam = c, by
 * backward substitution lam_i = (c_i - sum_{j>i} L_ji lam_j) / L_ii for
 * i = n-1..0, terms in ascending j (row i of L^T). */
void orc_trsv_upper_t(int n, const int32_t* rp, const int32_t* ci, const double* v,
                      const double* c, double* lam) {
  int nnz = rp[n];
  int32_t* trp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* tci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  orc_transpose(n, n, rp, ci, trp, tci, perm);
  for (int i = n - 1; i >= 0; --i) {
    double s = c[i];
    double d = 0.0;
    for (int q = trp[i]; q < trp[i + 1]; ++q) {
      int j = tci[q];
      if (j > i) s -= v[perm[q]] * lam[j];
      else if (j == i) d = v[perm[q]];
    }
    lam[i] = s / d;
  }
  free(trp); free(tci); free(perm);
}

/* Zero fill-in incomplete Cholesky, up-looking row form.  a holds the values
 * of lower(A) in the CSR pattern (rp, ci) (sorted, diagonal included); l
 * receives L in the same pattern.  For row i and each j in P_i, j < i in
 * ascending order:
 *     L_ij = (A_ij - sum_{k<j, k in P_i and P_j} L_ik L_jk) / L_jj
 * then d_i = A_ii - sum_{k<i} L_ik^2 and L_ii = sqrt(d_i).  Returns -1 on
 * success, else the first row whose d_i is not > 0 (that row's diagonal is
 * set to sqrt(d_i), possibly NaN, and the loop continues). */
int orc_ic0(int n, const int32_t* rp, const int32_t* ci, const double* a, double* l) {
  int fail = -1;
  for (int i = 0; i < n; ++i) {
    int pdiag = -1;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j == i) { pdiag = p; continue; }
      if (j > i) continue;
      double s = a[p];
      /* merge row i (positions before p) with row j (its off-diagonals) */
      int pi = rp[i], pj = rp[j];
      while (pi < p && pj < rp[j + 1]) {
        int ki = ci[pi], kj = ci[pj];
        if (kj >= j) break;
        if (ki == kj) { s -= l[pi] * l[pj]; ++pi; ++pj; }
        else if (ki < kj) ++pi;
        else ++pj;
      }
      /* L_jj is the diagonal of row j */
      double djj = 0.0;
      for (int q = rp[j]; q < rp[j + 1]; ++q) if (ci[q] == j) djj = l[q];
      l[p] = s / djj;
    }
    if (pdiag < 0) { if (fail < 0) fail = i; continue; }
    double d = a[pdiag];
    for (int p = rp[i]; p < rp[i + 1]; ++p) if (ci[p] < i) d -= l[p] * l[p];
    if (!(d > 0.0) && fail < 0) fail = i;
    l[pdiag] = sqrt(d);
  }
  return fail;
}

/* Zero fill-in incomplete LU by row-wise elimination on the pattern of A
 * (columns sorted in each row).  lu starts as a copy of a; for row i and each
 * stored k < i in ascending order: lu_ik /= u_kk, then lu_ij -= lu_ik * u_kj
 * for every stored j > k of row i whose (k, j) is stored.  Afterwards the
 * strictly lower part of lu is L (unit diagonal implied) and the rest is U.
 * Returns the first row whose pivot u_ii is zero, NaN or not stored, -1 if
 * none; elimination continues past it (its dependents get Inf/NaN). */
int orc_ilu0(int n, const int32_t* rp, const int32_t* ci, const double* a, double* lu) {
  int fail = -1;
  for (int p = 0; p < rp[n]; ++p) lu[p] = a[p];
  for (int i = 0; i < n; ++i) {
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int k = ci[p];
      if (k >= i) break;
      double ukk = 0.0;
      int pk = rp[k + 1];
      for (int q = rp[k]; q < rp[k + 1]; ++q) {
        if (ci[q] == k) ukk = lu[q];
        if (ci[q] > k) { pk = q; break; }
      }
      lu[p] = lu[p] / ukk;
      /* merge the rest of row i with the part of row k right of k */
      int pi = p + 1;
      while (pi < rp[i + 1] && pk < rp[k + 1]) {
        int ji = ci[pi], jk = ci[pk];
        if (ji == jk) { lu[pi] -= lu[p] * lu[pk]; ++pi; ++pk; }
        else if (ji < jk) ++pi;
        else ++pk;
      }
    }
    double d = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) if (ci[p] == i) d = lu[p];
    if (!(d != 0.0) && fail < 0) fail = i;
  }
  return fail;
}

/* Forward substitution with a unit-lower L stored as the strictly lower part
 * of a CSR matrix (other entries ignored): y_i = b_i - sum_{j<i} L_ij y_j. */
void orc_trsv_unit_lower(int n, const int32_t* rp, const int32_t* ci, const double* v,
                         const double* b, double* y) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p)
      if (ci[p] < i) s -= v[p] * y[ci[p]];
    y[i] = s;
  }
}

/* Gradients of loss = <w, A L^{-1} b>: given x = L^{-1} b and g = w,
 * lam = L^{-T} (A^T g), grad_b = lam and grad_L[p] = -lam_i x_j for every
 * stored (i, j) = p of L. */
void orc_backward(int n, int m, const int32_t* lrp, const int32_t* lci, const double* lv,
                  const int32_t* arp, const int32_t* aci, const double* av,
                  const double* x, const double* g, double* grad_b, double* grad_l) {
  double* c = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  orc_spmv_t(m, n, arp, aci, av, g, c);
  orc_trsv_upper_t(n, lrp, lci, lv, c, grad_b);
  for (int i = 0; i < n; ++i)
    for (int p = lrp[i]; p < lrp[i + 1]; ++p) grad_l[p] = -grad_b[i] * x[lci[p]];
  free(c);
}

/* Dependence levels of the SpTRSV DAG (wavefront number): level_i = 0 if row
 * i of L holds only its diagonal, else 1 + max over stored j < i of
 * level_j.  Returns the depth (number of levels), 0 for n = 0. */
int orc_levels(int n, const int32_t* rp, const int32_t* ci, int32_t* level) {
  int depth = 0;
  for (int i = 0; i < n; ++i) {
    int lv = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j < i && level[j] + 1 > lv) lv = level[j] + 1;
    }
    level[i] = lv;
    if (lv + 1 > depth) depth = lv + 1;
  }
  return depth;
}

/* Levels of the transposed (upper) solve: rlev_i = 0 if column i of L holds
 * only its diagonal, else 1 + max over stored L_ji with j > i of rlev_j. */
int orc_reverse_levels(int n, const int32_t* rp, const int32_t* ci, int32_t* rlev) {
  int nnz = rp[n];
  int32_t* trp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t* tci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  orc_transpose(n, n, rp, ci, trp, tci, perm);
  int depth = 0;
  for (int i = n - 1; i >= 0; --i) {
    int lv = 0;
    for (int q = trp[i]; q < trp[i + 1]; ++q) {
      int j = tci[q];
      if (j > i && rlev[j] + 1 > lv) lv = rlev[j] + 1;
    }
    rlev[i] = lv;
    if (lv + 1 > depth) depth = lv + 1;
  }
  free(trp); free(tci); free(perm);
  return depth;
}

/* Joint level of each SpMV row r in the SpTRSV -> SpMV pair, with F equal to
 * the pattern of A (row r of the product needs every x_j it reads):
 * ready_r = 1 + max_{j in A_r} level_j, and 0 for an empty row. */
void orc_spmv_ready(int m, const int32_t* arp, const int32_t* aci, const int32_t* level,
                    int32_t* ready) {
  for (int r = 0; r < m; ++r) {
    int lv = 0;
    for (int p = arp[r]; p < arp[r + 1]; ++p)
      if (level[aci[p]] + 1 > lv) lv = level[aci[p]] + 1;
    ready[r] = lv;
  }
}

/* Canonical joint order of the SpTRSV -> SpMV iteration set.  Iteration ids:
 * 0..n-1 are SpTRSV rows, n..n+m-1 are SpMV rows.  Sorted by (joint level,
 * SpTRSV before SpMV, row ascending).  Written by direct selection over
 * levels so that it is independent of any sorting routine. */
void orc_joint_order_ts(int n, const int32_t* level, int m, const int32_t* ready,
                        int32_t* order) {
  int maxlv = -1;
  for (int i = 0; i < n; ++i) if (level[i] > maxlv) maxlv = level[i];
  for (int r = 0; r < m; ++r) if (ready[r] > maxlv) maxlv = ready[r];
  int pos = 0;
  for (int lv = 0; lv <= maxlv; ++lv) {
    for (int i = 0; i < n; ++i) if (level[i] == lv) order[pos++] = i;
    for (int r = 0; r < m; ++r) if (ready[r] == lv) order[pos++] = n + r;
  }
}

/* Schedule validity for the SpTRSV -> SpMV pair.  order is a list of
 * iteration ids (see orc_joint_order_ts) cut into items by item_ptr.
 * Valid iff: order is a permutation of 0..n+m-1; item_ptr is a monotone
 * cover of it; and for every DAG edge u -> v (L_ij: j -> i for j < i;
 * A_rj: j -> n+r) u's item precedes v's item (strict: rows inside one item
 * must be independent), or, when allow_intra is set, u precedes v inside
 * the same item.  Returns 0 if valid, else a positive code naming the
 * first violated rule. */
int orc_validate_ts(int n, const int32_t* lrp, const int32_t* lci, int m,
                    const int32_t* arp, const int32_t* aci, const int32_t* order, int n_items,
                    const int32_t* item_ptr, int allow_intra) {
  int N = n + m;
  if (n_items < 0 || item_ptr[0] != 0 || item_ptr[n_items] != N) return 1;
  for (int t = 0; t < n_items; ++t) if (item_ptr[t + 1] <= item_ptr[t]) return 2;
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  int32_t* item = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  for (int u = 0; u < N; ++u) pos[u] = -1;
  for (int t = 0; t < n_items; ++t)
    for (int q = item_ptr[t]; q < item_ptr[t + 1]; ++q) {
      int u = order[q];
      if (u < 0 || u >= N || pos[u] >= 0) { free(pos); free(item); return 3; }
      pos[u] = q;
      item[u] = t;
    }
  int rc = 0;
  for (int i = 0; i < n && !rc; ++i)
    for (int p = lrp[i]; p < lrp[i + 1]; ++p) {
      int j = lci[p];
      if (j >= i) continue;
      int ok = item[j] < item[i] || (allow_intra && item[j] == item[i] && pos[j] < pos[i]);
      if (!ok) { rc = 4; break; }
    }
  for (int r = 0; r < m && !rc; ++r)
    for (int p = arp[r]; p < arp[r + 1]; ++p) {
      int j = aci[p], v = n + r;
      int ok = item[j] < item[v] || (allow_intra && item[j] == item[v] && pos[j] < pos[v]);
      if (!ok) { rc = 5; break; }
    }
  free(pos); free(item);
  return rc;
}

/* Schedule validity for a factorisation -> SpTRSV pair whose second kernel
 * reads only row i of the first at its row i (F = I: SpIC0 -> SpTRSV,
 * Table 2 combination 5, and SpILU0 -> SpTRSV, combination 6).  Iteration
 * ids: 0..n-1 are factor rows, n..2n-1 are solve rows.  Each stored entry
 * (i, j) with j < i of the factor's pattern is two edges, factor row j ->
 * factor row i (row i is eliminated against the final row j) and solve
 * row j -> solve row i (x_j is read); F = I adds factor row i -> solve row
 * i.  The iterations of one item run together, so an edge between two
 * items must go from an earlier item to a later one; the only edge allowed
 * inside an item is factor row i -> solve row i with the factor row listed
 * first (the interleaved packing of Sec. 2.3).  Valid iff order is a
 * permutation of 0..2n-1, item_ptr a cover of it by non-empty items, and
 * every edge is respected.  Returns 0 if valid, else a positive code naming
 * the first violated rule. */
int orc_validate_factor_solve(int n, const int32_t* rp, const int32_t* ci, const int32_t* order,
                              int n_items, const int32_t* item_ptr) {
  int N = 2 * n;
  if (n_items < 0 || item_ptr[0] != 0 || item_ptr[n_items] != N) return 1;
  for (int t = 0; t < n_items; ++t) if (item_ptr[t + 1] <= item_ptr[t]) return 2;
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  int32_t* item = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N > 0 ? N : 1));
  for (int u = 0; u < N; ++u) pos[u] = -1;
  for (int t = 0; t < n_items; ++t)
    for (int q = item_ptr[t]; q < item_ptr[t + 1]; ++q) {
      int u = order[q];
      if (u < 0 || u >= N || pos[u] >= 0) { free(pos); free(item); return 3; }
      pos[u] = q;
      item[u] = t;
    }
  int rc = 0;
  for (int i = 0; i < n && !rc; ++i) {
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      int j = ci[p];
      if (j >= i) continue;
      if (!(item[j] < item[i])) { rc = 4; break; }
      if (!(item[n + j] < item[n + i])) { rc = 5; break; }
    }
    if (!rc && !(item[i] < item[n + i] || (item[i] == item[n + i] && pos[i] < pos[n + i]))) rc = 6;
  }
  free(pos); free(item);
  return rc;
}

/* Validity of a static two-level schedule of the SpTRSV -> SpMV pair, as
 * a fused partitioning (Sec. 3.1) executes it: the nb s-partitions run one
 * after another, with a synchronisation between them; the w-partitions of
 * one s-partition are independent and run in parallel; the iterations of
 * one w-partition run in their listed order.  s_ptr (nb + 1 entries) cuts
 * the nw w-partitions into s-partitions, w_ptr (nw + 1 entries) cuts order
 * into w-partitions; empty partitions are allowed.  Valid iff the pointers
 * are monotone covers, order is a permutation of 0..n+m-1 (ids as in
 * orc_joint_order_ts), and every DAG edge u -> v (L_ij: j -> i for j < i;
 * A_rj: j -> n+r) has s(u) < s(v), or s(u) == s(v), w(u) == w(v) and u
 * listed before v.  Returns 0 if valid, else a positive code naming the
 * first violated rule. */
int orc_validate_static_ts(int n, const int32_t* lrp, const int32_t* lci, int m,
                           const int32_t* arp, const int32_t* aci, int nb, const int32_t* s_ptr,
                           int nw, const int32_t* w_ptr, const int32_t* order) {
  int N = n + m;
  if (nb < 0 || nw < 0 || s_ptr[0] != 0 || s_ptr[nb] != nw || w_ptr[0] != 0 || w_ptr[nw] != N) return 1;
  for (int b = 0; b < nb; ++b) if (s_ptr[b + 1] < s_ptr[b]) return 2;
  for (int w = 0; w < nw; ++w) if (w_ptr[w + 1] < w_ptr[w]) return 2;
  size_t cap = (size_t)(N > 0 ? N : 1);
  int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * cap);
  int32_t* wof = (int32_t*)malloc(sizeof(int32_t) * cap);
  int32_t* sof = (int32_t*)malloc(sizeof(int32_t) * cap);
  for (int u = 0; u < N; ++u) pos[u] = -1;
  int rc = 0;
  for (int b = 0; b < nb && !rc; ++b)
    for (int w = s_ptr[b]; w < s_ptr[b + 1] && !rc; ++w)
      for (int q = w_ptr[w]; q < w_ptr[w + 1]; ++q) {
        int u = order[q];
        if (u < 0 || u >= N || pos[u] >= 0) { rc = 3; break; }
        pos[u] = q;
        wof[u] = w;
        sof[u] = b;
      }
  /* an edge u -> v is respected if u's s-partition finishes first, or u
     runs earlier in the same w-partition */
#define ORC_BEFORE(u, v) (sof[u] < sof[v] || (wof[u] == wof[v] && pos[u] < pos[v]))
  for (int i = 0; i < n && !rc; ++i)
    for (int p = lrp[i]; p < lrp[i + 1]; ++p) {
      int j = lci[p];
      if (j >= i) continue;
      if (!ORC_BEFORE(j, i)) { rc = 4; break; }
    }
  for (int r = 0; r < m && !rc; ++r)
    for (int p = arp[r]; p < arp[r + 1]; ++p)
      if (!ORC_BEFORE(aci[p], n + r)) { rc = 5; break; }
#undef ORC_BEFORE
  free(pos); free(wof); free(sof);
  return rc;
}

/* Reuse ratio of the SpTRSV -> SpMV pair, from its stated form
 * 2 |x| / max(|A| + |x| + |y|, |L| + |x| + |b|) with sizes counted in
 * elements (nonzeros for matrices, lengths for vectors). */
double orc_reuse_ts(int n, int nnz_l, int m, int nnz_a) {
  double ka = (double)nnz_a + (double)n + (double)m;
  double kl = (double)nnz_l + (double)n + (double)n;
  return 2.0 * (double)n / (ka > kl ? ka : kl);
}

/* Reuse ratio of the SpIC0 -> SpTRSV pair (Table 2, combination 5):
 * 2 |L| / max(|L|, |L| + 2n). */
double orc_reuse_it(int n, int nnz_l) {
  double k1 = (double)nnz_l, k2 = (double)nnz_l + 2.0 * (double)n;
  return 2.0 * (double)nnz_l / (k1 > k2 ? k1 : k2);
}

/* Mixed-precision refinement of x = L^{-1} b with y = A x (one right-hand
 * side; FP32 solves, FP64 residuals), written stage by stage:
 *   x0   = the FP32 substitution of (L32, fl32(b));
 *   x    = 0 + (double) x0;
 *   for t = 1 .. ncorr:
 *     r   = b - L64 x          (FP64; row i sums its entries in ascending
 *                              column order from 0, diagonal last, then
 *                              subtracts the sum from b_i);
 *     d_t = the FP32 substitution of (L32, fl32(r));
 *     x   = x + (double) d_t   (FP64);
 *   y = A64 x                  (FP64, ascending, from 0);
 *   relres = max_i |b - L64 x|_i / max_i |b_i|  (0 / 0 reported as 0).
 * The FP32 substitution of (L32, c): for rows in order,
 *   s_i = sum over j < i ascending of fl32(L32_ij v_j), from 0 (FP32);
 *   v_i = fl32(fl32(c_i - s_i) / L32_ii).
 * stages (optional, n * (ncorr + 1) floats, row-major by row): row i's
 * x0_i, d_1i, ..., d_ncorr,i.  Returns relres. */
double orc_refine(int n, const int32_t* rp, const int32_t* ci, const double* l64, const float* l32,
                  int m, const int32_t* arp, const int32_t* aci, const double* a64,
                  const double* b, int ncorr, double* x, double* y, float* stages) {
  float* v = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  float* c = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
  double* r = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int t = 0; t <= ncorr; ++t) {
    /* right-hand side of this stage: fl32(b), then fl32(b - L64 x) */
    for (int i = 0; i < n; ++i) {
      if (t == 0) {
        c[i] = (float)b[i];
      } else {
        double acc = 0.0;
        for (int p = rp[i]; p < rp[i + 1]; ++p) acc += l64[p] * x[ci[p]];
        r[i] = b[i] - acc;
      }
    }
    if (t > 0)
      for (int i = 0; i < n; ++i) c[i] = (float)r[i];
    /* FP32 substitution */
    for (int i = 0; i < n; ++i) {
      float sum = 0.0f, dg = 0.0f;
      for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int j = ci[p];
        if (j < i) {
          float prod = l32[p] * v[j];
          sum = sum + prod;
        } else if (j == i) {
          dg = l32[p];
        }
      }
      float top = c[i] - sum;
      v[i] = top / dg;
    }
    for (int i = 0; i < n; ++i) {
      if (stages) stages[(size_t)i * (size_t)(ncorr + 1) + (size_t)t] = v[i];
      x[i] = (t == 0 ? 0.0 : x[i]) + (double)v[i];
    }
  }
  double rmax = 0.0, bmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) acc += l64[p] * x[ci[p]];
    double ri = b[i] - acc;
    if (fabs(ri) > rmax) rmax = fabs(ri);
    if (fabs(b[i]) > bmax) bmax = fabs(b[i]);
  }
  for (int i = 0; i < m; ++i) {
    double acc = 0.0;
    for (int p = arp[i]; p < arp[i + 1]; ++p) acc += a64[p] * x[aci[p]];
    y[i] = acc;
  }
  free(v);
  free(c);
  free(r);
  return bmax > 0.0 ? rmax / bmax : rmax;
}
