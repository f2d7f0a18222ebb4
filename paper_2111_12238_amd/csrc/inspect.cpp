// Host inspector: validation, dependence levels, the joint claim order,
// work items, transposes and SpIC0 intersection lists.
//
// Follows the paper's inspector (Sec. 2.2): the SpTRSV DAG is the pattern of
// L (a stored L_ij, j < i, is an edge j -> i), the inter-kernel dependence
// matrix F says which iterations of the first loop an iteration of the second
// loop needs (F = pattern(A) for a CSR SpMV reading x; F = I for SpIC0 ->
// SpTRSV), and the per-vertex cost is the number of nonzeros an iteration
// touches (Sec. 3.1).  Instead of the paper's multi-sparse DAG partitioning
// (LBC partitions, pairing, slack dispersion), the schedule is the joint
// DAG's wavefront order, claimed dynamically on the GPU: an SpMV row sits at
// the first wavefront where all x entries it reads are final, which fills
// the narrow SpTRSV wavefronts the way the paper's slack vertices do.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <limits>

#include "schedule.h"

namespace sf {

sf_status check_lower(const sf_csr_pattern* L) {
  if (!L || L->nrows < 0) return SF_ERR_ARG;
  if (L->nrows != L->ncols) return SF_ERR_SHAPE;
  const int32_t n = L->nrows;
  if (!L->rowptr) return SF_ERR_ARG;
  if (L->rowptr[0] != 0) return SF_ERR_CSR;
  if (n > 0 && !L->colind && L->rowptr[n] > 0) return SF_ERR_ARG;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t a = L->rowptr[i], b = L->rowptr[i + 1];
    if (b < a) return SF_ERR_CSR;
    for (int32_t p = a; p < b; ++p) {
      const int32_t j = L->colind[p];
      if (j < 0 || j >= n) return SF_ERR_CSR;
      if (p > a && L->colind[p - 1] >= j) return SF_ERR_CSR;
    }
  }
  // Shape checks after the structural ones so an unsorted row reports CSR.
  for (int32_t i = 0; i < n; ++i) {
    const int32_t a = L->rowptr[i], b = L->rowptr[i + 1];
    if (b > a && L->colind[b - 1] > i) return SF_ERR_NOT_LOWER;
    if (b == a || L->colind[b - 1] != i) return SF_ERR_ZERO_DIAG;
  }
  return SF_OK;
}

sf_status check_general(const sf_csr_pattern* A, int32_t ncols) {
  if (!A || A->nrows < 0 || !A->rowptr) return SF_ERR_ARG;
  if (A->ncols != ncols) return SF_ERR_SHAPE;
  if (A->rowptr[0] != 0) return SF_ERR_CSR;
  if (A->rowptr[A->nrows] > 0 && !A->colind) return SF_ERR_ARG;
  for (int32_t r = 0; r < A->nrows; ++r) {
    const int32_t a = A->rowptr[r], b = A->rowptr[r + 1];
    if (b < a) return SF_ERR_CSR;
    for (int32_t p = a; p < b; ++p) {
      const int32_t j = A->colind[p];
      if (j < 0 || j >= ncols) return SF_ERR_CSR;
      if (p > a && A->colind[p - 1] >= j) return SF_ERR_CSR;
    }
  }
  return SF_OK;
}

static void copy_pattern(Pattern& d, const sf_csr_pattern* s) {
  d.nrows = s->nrows;
  d.ncols = s->ncols;
  d.rp.assign(s->rowptr, s->rowptr + s->nrows + 1);
  const int64_t nnz = s->rowptr[s->nrows];
  d.ci.assign(s->colind, s->colind + nnz);
}

// CSR transpose; map[q] = source position of transposed entry q.
static void transpose(const Pattern& s, Pattern& t, std::vector<int32_t>& map) {
  t.nrows = s.ncols;
  t.ncols = s.nrows;
  t.rp.assign(size_t(t.nrows) + 1, 0);
  const int64_t nnz = s.nnz();
  for (int64_t p = 0; p < nnz; ++p) t.rp[s.ci[p] + 1]++;
  for (int32_t j = 0; j < t.nrows; ++j) t.rp[j + 1] += t.rp[j];
  t.ci.resize(nnz);
  map.resize(nnz);
  std::vector<int32_t> fill(t.rp.begin(), t.rp.end() - 1);
  for (int32_t i = 0; i < s.nrows; ++i)
    for (int32_t p = s.rp[i]; p < s.rp[i + 1]; ++p) {
      const int32_t q = fill[s.ci[p]]++;
      t.ci[q] = i;
      map[q] = p;
    }
}

// Stable counting sort of ids by an integer key in [0, nkeys).
static void counting_order(const std::vector<int32_t>& key, int32_t nkeys, std::vector<int32_t>& out) {
  std::vector<int64_t> cnt(size_t(nkeys) + 1, 0);
  for (int32_t k : key) cnt[k + 1]++;
  for (int32_t k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
  out.resize(key.size());
  for (size_t u = 0; u < key.size(); ++u) out[cnt[key[u]]++] = int32_t(u);
}

// Cut `order` into items: a new item starts when the (level, kind) key
// changes, when rows_per_item rows are reached, or when adding the next row
// would exceed the nonzero budget (a single row always fits).
static void cut_runs(const std::vector<int32_t>& order, const std::vector<int32_t>& key,
                     const std::vector<int32_t>& cost, int32_t rows_per_item, int32_t nnz_budget,
                     std::vector<int32_t>& item_ptr) {
  item_ptr.clear();
  item_ptr.push_back(0);
  const size_t N = order.size();
  size_t q = 0;
  while (q < N) {
    const int32_t k = key[order[q]];
    int64_t c = cost[order[q]];
    size_t e = q + 1;
    while (e < N && key[order[e]] == k && int32_t(e - q) < rows_per_item &&
           c + cost[order[e]] <= nnz_budget) {
      c += cost[order[e]];
      ++e;
    }
    item_ptr.push_back(int32_t(e));
    q = e;
  }
}

void cut_items(sf_schedule_s* s) {
  const int64_t n = s->n, m = s->m;
  if (s->kind == SF_TRSV_SPMV) {
    // Claim order: SpTRSV rows by level; an SpMV row (a slack iteration: any
    // slot at or after its joint level is valid) goes spmv_delay wavefronts
    // after the level where its inputs are final, so on the claim counters
    // it never gets ahead of the SpTRSV rows that form the critical path.
    // With spmv_delay = 0 this is the canonical joint order (joint level,
    // SpTRSV before SpMV, row).
    std::vector<int32_t> key(size_t(n + m)), cost(size_t(n + m));
    int32_t last = std::max(s->depth - 1, 0);
    for (int64_t r = 0; r < m; ++r) last = std::max(last, s->ready[r]);
    for (int64_t i = 0; i < n; ++i) {
      key[i] = 2 * s->level[i];
      cost[i] = std::max(1, s->L.rp[i + 1] - s->L.rp[i] - 1);
    }
    for (int64_t r = 0; r < m; ++r) {
      const int64_t slot = std::min<int64_t>(int64_t(s->ready[r]) + s->spmv_delay, last);
      key[n + r] = int32_t(2 * slot + 1);
      cost[n + r] = std::max(1, s->A.rp[r + 1] - s->A.rp[r]);
    }
    counting_order(key, 2 * (last + 1), s->order);
    cut_runs(s->order, key, cost, s->rows_per_item, s->max_item_nnz, s->item_ptr);
    s->trsv_items.clear();
    s->spmv_items.clear();
    for (size_t t = 0; t + 1 < s->item_ptr.size(); ++t) {
      if (s->order[s->item_ptr[t]] < n) s->trsv_items.push_back(int32_t(t));
      else s->spmv_items.push_back(int32_t(t));
    }
  } else {
    std::vector<int32_t> key(static_cast<size_t>(n)), cost(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
      key[i] = s->level[i];
      // SpIC0 row i touches its own row, the rows it reads and their pairs.
      int64_t c = 0;
      for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1]; ++p) c += 1 + (s->pair_ptr.empty() ? 0 : s->pair_ptr[p + 1] - s->pair_ptr[p]);
      cost[i] = int32_t(std::min<int64_t>(c, std::numeric_limits<int32_t>::max()));
    }
    cut_runs(s->order, key, cost, s->rows_per_item, s->max_item_nnz, s->item_ptr);
    s->trsv_items.clear();
    for (size_t t = 0; t + 1 < s->item_ptr.size(); ++t) s->trsv_items.push_back(int32_t(t));
  }
  // Level-set baseline: the SpTRSV items grouped by level.  Items are
  // level-pure, and in claim order the levels ascend.
  s->lvl_items = s->trsv_items;
  s->lvl_item_ptr.assign(size_t(s->depth) + 1, 0);
  for (int32_t t : s->lvl_items) {
    const int32_t row = s->order[s->item_ptr[t]];
    s->lvl_item_ptr[s->level[row] + 1]++;
  }
  for (int32_t l = 0; l < s->depth; ++l) s->lvl_item_ptr[l + 1] += s->lvl_item_ptr[l];
  // Backward items: runs of one reversed level.
  if (s->has_back) {
    std::vector<int32_t> key(static_cast<size_t>(n)), cost(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
      key[i] = s->rlevel[i];
      cost[i] = (s->LT.rp[i + 1] - s->LT.rp[i]) + (s->AT.rp[i + 1] - s->AT.rp[i]) +
                (s->L.rp[i + 1] - s->L.rp[i]);
    }
    cut_runs(s->border, key, cost, s->rows_per_item, s->max_item_nnz, s->bitem_ptr);
  }
}

static void build_pairs(sf_schedule_s* s) {
  const Pattern& L = s->L;
  const int64_t nnz = L.nnz();
  s->pair_ptr.assign(size_t(nnz) + 1, 0);
  s->pair_u.clear();
  s->pair_q.clear();
  for (int32_t i = 0; i < L.nrows; ++i) {
    const int32_t r0 = L.rp[i], rd = L.rp[i + 1] - 1;
    for (int32_t p = r0; p < rd; ++p) {
      const int32_t j = L.ci[p];
      int32_t pi = r0, pj = L.rp[j];
      const int32_t ej = L.rp[j + 1] - 1;  // row j's off-diagonals end here
      while (pi < p && pj < ej) {
        const int32_t ki = L.ci[pi], kj = L.ci[pj];
        if (ki == kj) {
          s->pair_u.push_back(((p - r0) << 16) | (pi - r0));  // (entry of row i, matching entry)
          s->pair_q.push_back(pj);
          ++pi;
          ++pj;
        } else if (ki < kj) {
          ++pi;
        } else {
          ++pj;
        }
      }
      s->pair_ptr[p + 1] = int32_t(s->pair_u.size());
    }
    s->pair_ptr[rd + 1] = int32_t(s->pair_u.size());  // the diagonal has no list
  }
}

sf_status build_schedule(sf_schedule_s* s, const sf_csr_pattern* Lp, const sf_csr_pattern* Ap,
                         const sf_inspect_opts& o) {
  s->kind = o.kind;
  copy_pattern(s->L, Lp);
  s->n = s->L.nrows;
  const int64_t n = s->n;
  if (s->kind == SF_TRSV_SPMV) {
    copy_pattern(s->A, Ap);
    s->m = s->A.nrows;
  } else {
    s->m = 0;
  }
  const int64_t m = s->m;

  // Levels (wavefront numbers) of the SpTRSV DAG.
  s->level.assign(size_t(n), 0);
  int32_t depth = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t lv = 0;
    for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1] - 1; ++p) lv = std::max(lv, s->level[s->L.ci[p]] + 1);
    s->level[i] = lv;
    depth = std::max(depth, lv + 1);
  }
  s->depth = depth;
  for (int64_t i = 0; i < n; ++i) s->max_offdiag = std::max(s->max_offdiag, s->L.rp[i + 1] - s->L.rp[i] - 1);
  {
    std::vector<int32_t> w(size_t(depth) + 1, 0);
    for (int32_t lv : s->level) w[lv]++;
    s->max_level_width = n ? *std::max_element(w.begin(), w.end()) : 0;
  }

  if (s->kind == SF_TRSV_SPMV) {
    // SpMV row r reads x_j for every stored A_rj (F = pattern of A): it can
    // run one wavefront after the last of them.
    s->ready.assign(size_t(m), 0);
    int32_t jd = depth;
    for (int64_t r = 0; r < m; ++r) {
      int32_t lv = 0;
      for (int32_t p = s->A.rp[r]; p < s->A.rp[r + 1]; ++p) lv = std::max(lv, s->level[s->A.ci[p]] + 1);
      s->ready[r] = lv;
      jd = std::max(jd, lv + 1);
    }
    s->joint_depth = jd;
    const double nn = double(n), mm = double(m);
    const double ka = double(s->A.nnz()) + nn + mm, kl = double(s->L.nnz()) + 2.0 * nn;
    s->reuse = (ka > 0 || kl > 0) ? 2.0 * nn / std::max(ka, kl) : 0.0;
  } else {
    s->joint_depth = depth;
    counting_order(s->level, std::max(depth, 1), s->order);
    const double nl = double(s->L.nnz());
    s->reuse = nl > 0 ? 2.0 * nl / std::max(nl, nl + 2.0 * double(n)) : 0.0;
    build_pairs(s);
  }

  if (o.want_backward && s->kind == SF_TRSV_SPMV) {
    s->has_back = true;
    transpose(s->L, s->LT, s->LT_map);
    transpose(s->A, s->AT, s->AT_map);
    // Reversed levels: rlev_i = 1 + max over stored L_ji, j > i, of rlev_j.
    s->rlevel.assign(size_t(n), 0);
    int32_t bd = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
      int32_t lv = 0;
      for (int32_t q = s->LT.rp[i] + 1; q < s->LT.rp[i + 1]; ++q) lv = std::max(lv, s->rlevel[s->LT.ci[q]] + 1);
      s->rlevel[i] = lv;
      bd = std::max(bd, lv + 1);
    }
    s->back_depth = bd;
    counting_order(s->rlevel, std::max(bd, 1), s->border);
  }

  // Default lanes per row from the mean row length (power of two, 2..32).
  auto pick = [](double mean) {
    int g = 2;
    while (g < 32 && g < mean) g *= 2;
    return g;
  };
  const double mean_l = n ? double(s->L.nnz() - n) / double(n) : 1.0;
  const double mean_a = m ? double(s->A.nnz()) / double(m) : 1.0;
  s->lanes_trsv = o.lanes_per_row > 0 ? o.lanes_per_row : pick(mean_l);
  s->lanes_spmv = std::max(4, pick(mean_a));  // SpMV kernels exist for 4..32 lanes
  if (s->kind == SF_IC0_TRSV) {
    // one lane per stored entry of an SpIC0 row
    int32_t maxlen = 1;
    for (int64_t i = 0; i < n; ++i) maxlen = std::max(maxlen, s->L.rp[i + 1] - s->L.rp[i]);
    int g = 4;
    while (g < 64 && g < maxlen) g *= 2;
    s->lanes_trsv = o.lanes_per_row > 0 ? o.lanes_per_row : g;
  }
  // one lane of a 64-wide wavefront finishes each row of an item
  s->rows_per_item = o.rows_per_item > 0 ? std::min(o.rows_per_item, 64) : 64;
  s->max_item_nnz = o.max_item_nnz > 0 ? o.max_item_nnz : 512;
  s->rhs_block = o.rhs_block;
  s->no_fusion = o.no_fusion;
  cut_items(s);
  return SF_OK;
}

int validate_forward(const sf_schedule_s* s) {
  const int64_t n = s->n, m = s->m;
  const int64_t N = s->kind == SF_TRSV_SPMV ? n + m : n;
  std::vector<int32_t> item(size_t(N), -1);
  const int64_t nitems = int64_t(s->item_ptr.size()) - 1;
  if (s->item_ptr.empty() || s->item_ptr[0] != 0 || s->item_ptr.back() != N) return 1;
  for (int64_t t = 0; t < nitems; ++t) {
    if (s->item_ptr[t + 1] <= s->item_ptr[t]) return 2;
    for (int32_t q = s->item_ptr[t]; q < s->item_ptr[t + 1]; ++q) {
      const int32_t u = s->order[q];
      if (u < 0 || u >= N || item[u] >= 0) return 3;
      item[u] = int32_t(t);
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1] - 1; ++p)
      if (!(item[s->L.ci[p]] < item[i])) return 4;
  if (s->kind == SF_TRSV_SPMV)
    for (int64_t r = 0; r < m; ++r)
      for (int32_t p = s->A.rp[r]; p < s->A.rp[r + 1]; ++p)
        if (!(item[s->A.ci[p]] < item[n + r])) return 5;
  return 0;
}

}  // namespace sf
