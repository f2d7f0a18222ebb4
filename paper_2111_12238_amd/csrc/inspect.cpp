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
#include <queue>
#include <utility>

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

// SpILU0 input: a square CSR pattern with sorted columns and a stored
// diagonal in every row.
sf_status check_square_diag(const sf_csr_pattern* A) {
  if (!A || A->nrows < 0) return SF_ERR_ARG;
  if (A->nrows != A->ncols) return SF_ERR_SHAPE;
  const sf_status st = check_general(A, A->ncols);
  if (st != SF_OK) return st;
  for (int32_t i = 0; i < A->nrows; ++i) {
    const int32_t* b = A->colind + A->rowptr[i];
    const int32_t* e = A->colind + A->rowptr[i + 1];
    if (!std::binary_search(b, e, i)) return SF_ERR_ZERO_DIAG;
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
// would exceed the nonzero budget (a single row always fits).  Runs of odd
// keys (SpMV rows of the joint order) may take `odd_scale` times the rows
// (at most 64) and the budget.
static void cut_runs(const std::vector<int32_t>& order, const std::vector<int32_t>& key,
                     const std::vector<int32_t>& cost, int32_t rows_per_item, int32_t nnz_budget,
                     std::vector<int32_t>& item_ptr, int32_t odd_scale = 1) {
  item_ptr.clear();
  item_ptr.push_back(0);
  const size_t N = order.size();
  size_t q = 0;
  while (q < N) {
    const int32_t k = key[order[q]];
    const bool odd = (k & 1) != 0 && odd_scale > 1;
    const int32_t rows = odd ? std::min(64, rows_per_item * odd_scale) : rows_per_item;
    const int64_t budget = odd ? int64_t(nnz_budget) * odd_scale : int64_t(nnz_budget);
    int64_t c = cost[order[q]];
    size_t e = q + 1;
    while (e < N && key[order[e]] == k && int32_t(e - q) < rows && c + cost[order[e]] <= budget) {
      c += cost[order[e]];
      ++e;
    }
    item_ptr.push_back(int32_t(e));
    q = e;
  }
}

// Critical-path model used to choose between the two plans: a dependence
// between items costs about one device-coherent round trip plus the item's
// load round (kEstHop), and each wavefront inside an item one LDS-staged
// step (kEstStep).  Both constants are rough MI355X measurements; the
// autotuner times the two plans when the estimate is not trusted.
constexpr double kEstHop = 1.5, kEstStep = 0.15;

// Coarsened items by locality-greedy topological ordering.  Rows are taken
// one at a time in a topological order (Kahn's algorithm); the current item
// grows with the ready row that has the most predecessors already in it
// (ties: lower level, then lower row), and closes at R rows, at the entry
// budget, or when no ready row touches it.  A new item starts from the
// lowest-level ready row.  Every item is a contiguous run of one
// topological order, so every DAG edge goes from an item to itself or to a
// later item.  On meshes this grows compact blocks whose internal chains
// replace many dependent wavefronts.
//
// The DAG: row i's predecessors are ci[p] for p in [rp[i] + lo, rp[i+1] - hi)
// (lo = 1, hi = 0 when the diagonal is stored first; lo = 0, hi = 1 when
// last).  Item rows come out sorted by (local wavefront, row).
struct ChunkPlan {
  std::vector<int32_t> rows, ptr, chunk_of, slot;  // rows in item order; item boundaries
  std::vector<uint8_t> lloc;                       // local wavefront per row (indexed by row)
  std::vector<double> cp;                          // critical-path estimate at each item's end
  int32_t chain = 0, maxloc = 0;
  double cp_max = 0.0;
};

static ChunkPlan chunk_dag(int32_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, int lo,
                           int hi, const std::vector<int32_t>& level, int32_t R, int64_t budget) {
  ChunkPlan c;
  auto pb = [&](int32_t i) { return rp[i] + lo; };
  auto pe = [&](int32_t i) { return rp[i + 1] - hi; };
  std::vector<int32_t> sp(size_t(n) + 1, 0), si;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t p = pb(i); p < pe(i); ++p) sp[size_t(ci[p]) + 1]++;
  for (int32_t i = 0; i < n; ++i) sp[size_t(i) + 1] += sp[i];
  si.resize(size_t(sp[n]));
  {
    std::vector<int32_t> fill(sp.begin(), sp.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t p = pb(i); p < pe(i); ++p) si[size_t(fill[ci[p]]++)] = i;
  }
  std::vector<int32_t> indeg(static_cast<size_t>(n)), score(static_cast<size_t>(n), 0), touched;
  c.chunk_of.assign(size_t(n), -1);
  c.lloc.assign(size_t(n), 0);
  using Key = std::pair<int64_t, int32_t>;  // (level, row)
  std::priority_queue<Key, std::vector<Key>, std::greater<Key>> ready;
  for (int32_t i = 0; i < n; ++i) {
    indeg[i] = pe(i) - pb(i);
    if (indeg[i] == 0) ready.push({level[i], i});
  }
  struct Cand {
    int32_t score, level, row;
    bool operator<(const Cand& o) const {  // max-heap: more predecessors inside, then lower level, row
      if (score != o.score) return score < o.score;
      if (level != o.level) return level > o.level;
      return row > o.row;
    }
  };
  std::priority_queue<Cand> cand;
  c.rows.reserve(size_t(n));
  c.ptr.push_back(0);
  int32_t cid = 0;
  int64_t done = 0;
  auto cost_of = [&](int32_t i) { return int64_t(std::max(1, pe(i) - pb(i))); };
  auto add = [&](int32_t u) {
    c.chunk_of[u] = cid;
    int32_t d = 0;
    for (int32_t p = pb(u); p < pe(u); ++p)
      if (c.chunk_of[ci[p]] == cid) d = std::max<int32_t>(d, c.lloc[ci[p]] + 1);
    c.lloc[u] = uint8_t(d);
    c.rows.push_back(u);
    ++done;
    for (int32_t q = sp[u]; q < sp[u + 1]; ++q) {
      const int32_t v = si[q];
      if (score[v] == 0) touched.push_back(v);
      ++score[v];
      if (--indeg[v] == 0) {
        ready.push({level[v], v});
        cand.push({score[v], level[v], v});
      }
    }
  };
  while (done < n) {
    while (c.chunk_of[ready.top().second] >= 0) ready.pop();
    const int32_t seed = ready.top().second;
    ready.pop();
    int64_t cost = cost_of(seed);
    int32_t size = 1;
    add(seed);
    while (size < R && !cand.empty()) {
      const Cand k = cand.top();
      if (c.chunk_of[k.row] >= 0 || score[k.row] != k.score) {  // stale heap entry
        cand.pop();
        continue;
      }
      if (cost + cost_of(k.row) > budget) break;
      {  // local wavefronts are kept in a byte: an item closes before its 255th
        int32_t d = 0;
        for (int32_t p = pb(k.row); p < pe(k.row); ++p)
          if (c.chunk_of[ci[p]] == cid) d = std::max<int32_t>(d, c.lloc[ci[p]] + 1);
        if (d >= 255) break;
      }
      cand.pop();
      cost += cost_of(k.row);
      ++size;
      add(k.row);
    }
    for (int32_t v : touched) score[v] = 0;
    touched.clear();
    cand = std::priority_queue<Cand>();
    c.ptr.push_back(int32_t(c.rows.size()));
    ++cid;
  }
  const int32_t nc = cid;
  c.slot.assign(size_t(n), 0);
  for (int32_t k = 0; k < nc; ++k) {
    auto b = c.rows.begin() + c.ptr[k], e = c.rows.begin() + c.ptr[k + 1];
    std::sort(b, e, [&](int32_t x, int32_t y) { return c.lloc[x] != c.lloc[y] ? c.lloc[x] < c.lloc[y] : x < y; });
    for (int32_t q = c.ptr[k]; q < c.ptr[k + 1]; ++q) {
      c.slot[c.rows[q]] = q - c.ptr[k];
      c.maxloc = std::max<int32_t>(c.maxloc, c.lloc[c.rows[q]]);
    }
  }
  // Critical-path estimate over the item graph (item ids are topological).
  c.cp.assign(size_t(nc), 0.0);
  std::vector<int32_t> chain(size_t(nc), 1);
  for (int32_t k = 0; k < nc; ++k) {
    double in = 0.0;
    int32_t ch = 0, depth_k = 0;
    for (int32_t q = c.ptr[k]; q < c.ptr[k + 1]; ++q) {
      const int32_t u = c.rows[q];
      depth_k = std::max<int32_t>(depth_k, c.lloc[u] + 1);
      for (int32_t p = pb(u); p < pe(u); ++p) {
        const int32_t pc = c.chunk_of[ci[p]];
        if (pc != k) {
          in = std::max(in, c.cp[pc]);
          ch = std::max(ch, chain[pc]);
        }
      }
    }
    c.cp[k] = in + kEstHop + kEstStep * depth_k;
    chain[k] = ch + 1;
    c.cp_max = std::max(c.cp_max, c.cp[k]);
    c.chain = std::max(c.chain, chain[k]);
  }
  return c;
}

// Critical-path model of items whose rows wait for their own inputs
// (pipelined items): an item runs its local wavefronts in order, each in
// batches of up to 64 rows costing kPipeStep, and a local wavefront starts
// once the previous one is done and every input from another item has been
// published for kPipeHop.  Measured on MI355X: with the coarsened plan's
// 64-row items on the 3D 7-point 128^3 grid the model gives 434 us against
// 459 us measured.
constexpr double kPipeHop = 3.8, kPipeStep = 0.21;

static double pipelined_estimate(int32_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, int lo,
                                 int hi, const ChunkPlan& c) {
  std::vector<double> trow(size_t(n), 0.0);
  double tmax = 0.0;
  const int32_t nc = int32_t(c.ptr.size()) - 1;
  for (int32_t k = 0; k < nc; ++k) {
    double fin = 0.0;
    int32_t q = c.ptr[k];
    while (q < c.ptr[k + 1]) {
      const int32_t lv = c.lloc[c.rows[q]];
      int32_t e = q;
      while (e < c.ptr[k + 1] && c.lloc[c.rows[e]] == lv) ++e;
      double start = fin;
      for (int32_t t = q; t < e; ++t) {
        const int32_t u = c.rows[t];
        for (int32_t p = rp[u] + lo; p < rp[u + 1] - hi; ++p)
          if (c.chunk_of[ci[p]] != k) start = std::max(start, trow[ci[p]] + kPipeHop);
      }
      fin = start + kPipeStep * double((e - q + 63) / 64);
      for (int32_t t = q; t < e; ++t) trow[c.rows[t]] = fin;
      q = e;
    }
    tmax = std::max(tmax, fin);
  }
  return tmax;
}

// Per stored entry p of a row: the slot of its column inside the row's item,
// or 0xFF (other item, or the diagonal).
static std::vector<uint8_t> entry_slots(const ChunkPlan& c, int32_t n, const std::vector<int32_t>& rp,
                                        const std::vector<int32_t>& ci, int lo, int hi) {
  std::vector<uint8_t> e(rp.empty() ? 0 : size_t(rp[n]), 0xFF);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t p = rp[i] + lo; p < rp[i + 1] - hi; ++p)
      if (c.chunk_of[ci[p]] == c.chunk_of[i]) e[size_t(p)] = uint8_t(c.slot[ci[p]]);
  return e;
}

// Forward coarsened plan: SpTRSV items from chunk_dag over L; SpMV rows
// follow the item holding their last input (plus the slack delay, in items
// of a typical chain step).
static void build_chunks(sf_schedule_s* s) {
  const Pattern& L = s->L;
  const int32_t n = L.nrows;
  const int64_t m = s->m;
  const int32_t R = std::max(1, std::min(s->rows_per_item, 64));
  const int64_t budget = std::min<int64_t>(s->max_item_nnz, kChunkEntries);
  const ChunkPlan c = chunk_dag(n, L.rp, L.ci, 0, 1, s->level, R, budget);
  const int32_t nc = int32_t(c.ptr.size()) - 1;
  std::vector<int32_t> skey(size_t(m), -1);
  double cp_all = c.cp_max;
  for (int64_t r = 0; r < m; ++r) {
    double in = 0.0;
    for (int32_t p = s->A.rp[r]; p < s->A.rp[r + 1]; ++p) {
      const int32_t k = c.chunk_of[s->A.ci[p]];
      skey[r] = std::max(skey[r], k);
      in = std::max(in, c.cp[k]);
    }
    cp_all = std::max(cp_all, in + kEstHop);
  }
  // by default SpMV rows go after every SpTRSV item here: interleaved with
  // coarsened items they take wavefronts and memory bandwidth from the
  // critical chain
  const int64_t delay = s->spmv_delay < 0 ? (int64_t(1) << 30) : int64_t(s->spmv_delay);
  if (delay > 0 && nc > 0) {
    const int64_t per_step = std::max<int64_t>(1, nc / std::max(1, c.chain));
    for (int64_t r = 0; r < m; ++r)
      skey[r] = int32_t(std::min<int64_t>(int64_t(skey[r]) + delay * per_step, nc - 1));
  }
  // Claim order: [SpMV rows without inputs] item 0, its SpMV rows, item 1, ...
  std::vector<int32_t> bucket(static_cast<size_t>(nc) + 2, 0), sorder(static_cast<size_t>(m));
  for (int64_t r = 0; r < m; ++r) bucket[size_t(skey[r] + 1) + 1]++;
  for (size_t k = 0; k + 1 < bucket.size(); ++k) bucket[k + 1] += bucket[k];
  {
    std::vector<int32_t> fill(bucket.begin(), bucket.end() - 1);
    for (int64_t r = 0; r < m; ++r) sorder[size_t(fill[size_t(skey[r] + 1)]++)] = int32_t(r);
  }
  s->corder.clear();
  s->citem_ptr.assign(1, 0);
  s->ctrsv_items.clear();
  s->clloc.clear();
  s->corder.reserve(size_t(n + m));
  s->clloc.reserve(size_t(n + m));
  auto spmv_run = [&](int32_t b) {  // SpMV rows of bucket b, cut by rows and budget
    int32_t q = bucket[b];
    const int32_t e = bucket[b + 1];
    while (q < e) {
      int64_t cost = 0;
      int32_t k = q;
      while (k < e && k - q < R) {
        const int32_t r = sorder[k];
        const int64_t cr = std::max(1, s->A.rp[r + 1] - s->A.rp[r]);
        if (k > q && cost + cr > s->max_item_nnz) break;
        cost += cr;
        ++k;
      }
      for (int32_t t = q; t < k; ++t) {
        s->corder.push_back(int32_t(n + sorder[t]));
        s->clloc.push_back(0);
      }
      s->citem_ptr.push_back(int32_t(s->corder.size()));
      q = k;
    }
  };
  spmv_run(0);
  for (int32_t k = 0; k < nc; ++k) {
    for (int32_t q = c.ptr[k]; q < c.ptr[k + 1]; ++q) {
      s->corder.push_back(c.rows[q]);
      s->clloc.push_back(c.lloc[c.rows[q]]);
    }
    s->ctrsv_items.push_back(int32_t(s->citem_ptr.size()) - 1);
    s->citem_ptr.push_back(int32_t(s->corder.size()));
    spmv_run(k + 1);
  }
  s->celoc = entry_slots(c, n, L.rp, L.ci, 0, 1);
  s->est_chunk_pipe_us = pipelined_estimate(n, L.rp, L.ci, 0, 1, c);
  s->chunk_chain = c.chain;
  s->max_local_depth = nc > 0 ? c.maxloc + 1 : 0;
  s->est_chunk_us = cp_all;
}

// Region plan (one wavefront per region, regions of up to region_rows rows
// grown by chunk_dag without an entry budget).  A region's rows run level
// by level inside one wavefront, each local level in batches of up to 64
// rows, with the region's x values kept in LDS; every row waits only for its
// own inputs, so a region starts as soon as its first rows' inputs exist
// and regions downstream overlap the ones they depend on.  Per region: its
// batches (first position, first external input first used there), its
// external inputs (distinct columns read from other regions, in order of
// first use) and, per stored off-diagonal of its rows, a 16-bit code: the
// column's position inside the region, or 0x8000 | the external input's
// index.  Per position the offset of its row's entries inside the region's
// entry table.  SpMV rows follow as in the coarsened plan.
static void build_regions(sf_schedule_s* s, int32_t rows) {
  const Pattern& L = s->L;
  const int32_t n = L.nrows;
  const int64_t m = s->m;
  const int32_t R = std::max(64, std::min(rows, 16384));
  const ChunkPlan c = chunk_dag(n, L.rp, L.ci, 0, 1, s->level, R, int64_t(1) << 62);
  const int32_t nc = int32_t(c.ptr.size()) - 1;
  // SpMV rows after the region holding their last input, by default after every region
  std::vector<int32_t> skey(size_t(m), -1);
  for (int64_t r = 0; r < m; ++r)
    for (int32_t p = s->A.rp[r]; p < s->A.rp[r + 1]; ++p) skey[r] = std::max(skey[r], c.chunk_of[s->A.ci[p]]);
  const int64_t delay = s->spmv_delay < 0 ? (int64_t(1) << 30) : int64_t(s->spmv_delay);
  if (delay > 0 && nc > 0) {
    const int64_t per_step = std::max<int64_t>(1, nc / std::max(1, c.chain));
    for (int64_t r = 0; r < m; ++r)
      skey[r] = int32_t(std::min<int64_t>(int64_t(skey[r]) + delay * per_step, nc - 1));
  }
  std::vector<int32_t> bucket(static_cast<size_t>(nc) + 2, 0), sorder(static_cast<size_t>(m));
  for (int64_t r = 0; r < m; ++r) bucket[size_t(skey[r] + 1) + 1]++;
  for (size_t k = 0; k + 1 < bucket.size(); ++k) bucket[k + 1] += bucket[k];
  {
    std::vector<int32_t> fill(bucket.begin(), bucket.end() - 1);
    for (int64_t r = 0; r < m; ++r) sorder[size_t(fill[size_t(skey[r] + 1)]++)] = int32_t(r);
  }
  s->rorder.clear();
  s->ritem_ptr.assign(1, 0);
  s->rtrsv_items.clear();
  s->rlloc.clear();
  s->rroff.clear();
  s->rbatch.clear();           // pairs (first position, first external index) per batch
  s->rbatch_ptr.assign(1, 0);  // per item: its batches
  s->rext.clear();
  s->rext_ptr.assign(1, 0);    // per item: its external inputs
  s->rcode.assign(size_t(L.nnz()), 0);
  s->region_rows_max = s->region_entries_max = s->region_ext_max = s->region_batches_max = 0;
  auto close_item = [&]() {
    s->ritem_ptr.push_back(int32_t(s->rorder.size()));
    s->rbatch_ptr.push_back(int32_t(s->rbatch.size() / 2));
    s->rext_ptr.push_back(int32_t(s->rext.size()));
  };
  // SpMV items of up to 256 rows (64 per wavefront and pass) and at least
  // 2048 entries of budget: they run after the regions, where fewer, larger
  // items measured faster (128^3: 0.38 -> 0.33 ms against 128-row items)
  const int64_t spmv_budget = std::max<int64_t>(s->max_item_nnz, 2048);
  auto spmv_run = [&](int32_t b) {  // SpMV rows of bucket b
    int32_t q = bucket[b];
    const int32_t e = bucket[b + 1];
    while (q < e) {
      int64_t cost = 0;
      int32_t k = q;
      while (k < e && k - q < 256) {
        const int32_t r = sorder[k];
        const int64_t cr = std::max(1, s->A.rp[r + 1] - s->A.rp[r]);
        if (k > q && cost + cr > spmv_budget) break;
        cost += cr;
        ++k;
      }
      for (int32_t t = q; t < k; ++t) {
        s->rorder.push_back(int32_t(n + sorder[t]));
        s->rlloc.push_back(0);
        s->rroff.push_back(0);
      }
      close_item();
      q = k;
    }
  };
  std::vector<int32_t> ext_of(size_t(n), -1), ext_stamp(size_t(n), -1);
  spmv_run(0);
  for (int32_t k = 0; k < nc; ++k) {
    const int32_t q0 = int32_t(s->rorder.size());
    const int32_t e0 = int32_t(s->rext.size());
    int32_t overflow = 0;  // entries past each row's first kRegionAhead
    for (int32_t q = c.ptr[k]; q < c.ptr[k + 1]; ++q) {
      const int32_t u = c.rows[q];
      const int32_t pos = int32_t(s->rorder.size());
      // a new batch at a change of local level or every 64 rows of one level
      if (q == c.ptr[k] || c.lloc[u] != c.lloc[c.rows[q - 1]] || (pos - s->rbatch[s->rbatch.size() - 2]) >= 64) {
        s->rbatch.push_back(pos);
        s->rbatch.push_back(int32_t(s->rext.size()) - e0);
      }
      s->rorder.push_back(u);
      s->rlloc.push_back(c.lloc[u]);
      s->rroff.push_back(overflow);
      for (int32_t p = L.rp[u]; p < L.rp[u + 1] - 1; ++p) {
        const int32_t j = L.ci[p];
        if (c.chunk_of[j] == k) {
          s->rcode[size_t(p)] = uint16_t(c.slot[j]);
        } else {
          if (ext_stamp[j] != k) {
            ext_stamp[j] = k;
            ext_of[j] = int32_t(s->rext.size()) - e0;
            s->rext.push_back(j);
          }
          s->rcode[size_t(p)] = uint16_t(0x8000 | ext_of[j]);
        }
      }
      overflow += std::max(0, L.rp[u + 1] - 1 - L.rp[u] - kRegionAhead);
    }
    s->rtrsv_items.push_back(int32_t(s->ritem_ptr.size()) - 1);
    s->region_rows_max = std::max(s->region_rows_max, int32_t(s->rorder.size()) - q0);
    s->region_entries_max = std::max(s->region_entries_max, overflow);
    s->region_ext_max = std::max(s->region_ext_max, int32_t(s->rext.size()) - e0);
    close_item();
    const size_t nbp = s->rbatch_ptr.size();
    s->region_batches_max = std::max(s->region_batches_max, s->rbatch_ptr[nbp - 1] - s->rbatch_ptr[nbp - 2]);
    spmv_run(k + 1);
  }
  s->rbatch.push_back(int32_t(s->rorder.size()));  // end sentinel: the last batch's end
  s->rbatch.push_back(0);
  s->region_chain = c.chain;
  s->est_region_us = pipelined_estimate(n, L.rp, L.ci, 0, 1, c);
}

// Backward coarsened plan: chunk_dag over L^T (the transposed solve's
// predecessors of row i are the rows j > i with L_ji stored; the diagonal is
// stored first in each row of L^T).
// Backward region plan: regions of up to `rows` rows over the transposed
// solve's DAG (rows of L^T, predecessors j > i with L_ji stored, diagonal
// first in each row of L^T), laid out as the forward region plan
// (build_regions) without SpMV rows.  brcode is indexed by L^T position.
static void build_back_regions(sf_schedule_s* s, int32_t rows) {
  const int32_t n = int32_t(s->n);
  const int32_t R = std::max(64, std::min(rows, 1024));
  const ChunkPlan c = chunk_dag(n, s->LT.rp, s->LT.ci, 1, 0, s->rlevel, R, int64_t(1) << 62);
  const int32_t nc = int32_t(c.ptr.size()) - 1;
  s->brorder.clear();
  s->britem_ptr.assign(1, 0);
  s->brlloc.clear();
  s->brroff.clear();
  s->brbatch.clear();
  s->brbatch_ptr.assign(1, 0);
  s->brext.clear();
  s->brext_ptr.assign(1, 0);
  s->brcode.assign(size_t(s->LT.nnz()), 0);
  s->back_region_rows_max = s->back_region_entries_max = s->back_region_ext_max = s->back_region_batches_max = 0;
  std::vector<int32_t> ext_of(size_t(n), -1), ext_stamp(size_t(n), -1);
  for (int32_t k = 0; k < nc; ++k) {
    const int32_t q0 = int32_t(s->brorder.size());
    const int32_t e0 = int32_t(s->brext.size());
    int32_t overflow = 0;
    for (int32_t q = c.ptr[k]; q < c.ptr[k + 1]; ++q) {
      const int32_t u = c.rows[q];
      const int32_t pos = int32_t(s->brorder.size());
      if (q == c.ptr[k] || c.lloc[u] != c.lloc[c.rows[q - 1]] || (pos - s->brbatch[s->brbatch.size() - 2]) >= 64) {
        s->brbatch.push_back(pos);
        s->brbatch.push_back(int32_t(s->brext.size()) - e0);
      }
      s->brorder.push_back(u);
      s->brlloc.push_back(c.lloc[u]);
      s->brroff.push_back(overflow);
      for (int32_t p = s->LT.rp[u] + 1; p < s->LT.rp[u + 1]; ++p) {
        const int32_t j = s->LT.ci[p];
        if (c.chunk_of[j] == k) {
          s->brcode[size_t(p)] = uint16_t(c.slot[j]);
        } else {
          if (ext_stamp[j] != k) {
            ext_stamp[j] = k;
            ext_of[j] = int32_t(s->brext.size()) - e0;
            s->brext.push_back(j);
          }
          s->brcode[size_t(p)] = uint16_t(0x8000 | ext_of[j]);
        }
      }
      overflow += std::max(0, s->LT.rp[u + 1] - 1 - s->LT.rp[u] - kRegionAhead);
    }
    s->back_region_rows_max = std::max(s->back_region_rows_max, int32_t(s->brorder.size()) - q0);
    s->back_region_entries_max = std::max(s->back_region_entries_max, overflow);
    s->back_region_ext_max = std::max(s->back_region_ext_max, int32_t(s->brext.size()) - e0);
    s->britem_ptr.push_back(int32_t(s->brorder.size()));
    s->brbatch_ptr.push_back(int32_t(s->brbatch.size() / 2));
    s->brext_ptr.push_back(int32_t(s->brext.size()));
    const size_t nbp = s->brbatch_ptr.size();
    s->back_region_batches_max = std::max(s->back_region_batches_max, s->brbatch_ptr[nbp - 1] - s->brbatch_ptr[nbp - 2]);
  }
  s->brbatch.push_back(int32_t(s->brorder.size()));  // end sentinel
  s->brbatch.push_back(0);
  s->back_region_chain = c.chain;
  s->est_back_region_us = pipelined_estimate(n, s->LT.rp, s->LT.ci, 1, 0, c);
}

static void build_back_chunks(sf_schedule_s* s) {
  const int32_t n = int32_t(s->n);
  const int32_t R = std::max(1, std::min(s->rows_per_item, 64));
  const int64_t budget = std::min<int64_t>(s->max_item_nnz, kChunkEntries);
  const ChunkPlan c = chunk_dag(n, s->LT.rp, s->LT.ci, 1, 0, s->rlevel, R, budget);
  s->bcorder = c.rows;
  s->bcitem_ptr = c.ptr;
  s->bclloc.resize(size_t(n));
  for (int32_t q = 0; q < n; ++q) s->bclloc[q] = c.lloc[c.rows[q]];
  s->bceloc = entry_slots(c, n, s->LT.rp, s->LT.ci, 1, 0);
  s->back_chunk_chain = c.chain;
  s->est_back_chunk_us = c.cp_max;
  s->est_back_chunk_pipe_us = pipelined_estimate(n, s->LT.rp, s->LT.ci, 1, 0, c);
}

// Fraction test of the auto mode: coarsening pays where most edges join
// consecutive wavefronts (mesh-like DAGs, whose chains a compact item can
// absorb); on DAGs whose edges skip many wavefronts it is not estimated.
static bool mesh_like(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, int lo, int hi,
                      const std::vector<int32_t>& level) {
  int64_t tight = 0, edges = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = rp[i] + lo; p < rp[i + 1] - hi; ++p) {
      ++edges;
      tight += level[i] == level[ci[p]] + 1;
    }
  return edges > 0 && double(tight) >= 0.35 * double(edges);
}

// Row ranges per claim position (see sf_schedule_s::qrng); SpIC0 schedules
// get the SpTRSV ranges of their rows.
static void position_ranges(const sf_schedule_s* s, const std::vector<int32_t>& order, std::vector<int32_t>& out) {
  out.resize(2 * order.size());
  for (size_t q = 0; q < order.size(); ++q) {
    const int32_t id = order[q];
    if (id < s->n) {
      out[2 * q] = s->L.rp[id];
      out[2 * q + 1] = s->L.rp[id + 1] - 1;
    } else {
      out[2 * q] = s->A.rp[id - s->n];
      out[2 * q + 1] = s->A.rp[id - s->n + 1];
    }
  }
}

// Prefix fusion (sf_schedule_s::apre, pqrng) over the level plan's claim
// order: row r qualifies when A's row r starts with exactly L's row r
// off-diagonal columns followed by the diagonal.  Its SpMV row then comes
// after SpTRSV row r in claim order (it reads x_r), which the fold's
// hand-over needs.
static void prefix_ranges(sf_schedule_s* s) {
  s->apre.clear();
  s->pqrng.clear();
  s->prefix_rows = 0;
  s->prefix_entries = 0;
  if (s->kind != SF_TRSV_SPMV || s->m == 0 || s->A.rp.empty()) return;
  const int64_t n = s->n, lim = std::min<int64_t>(s->n, s->m);
  std::vector<int32_t> pre(size_t(lim), 0);
  for (int64_t r = 0; r < lim; ++r) {
    const int32_t l0 = s->L.rp[r], cnt = s->L.rp[r + 1] - 1 - l0, a0 = s->A.rp[r];
    if (s->A.rp[r + 1] - a0 < cnt + 1) continue;
    bool ok = s->A.ci[size_t(a0 + cnt)] == r;
    for (int32_t t = 0; ok && t < cnt; ++t) ok = s->A.ci[size_t(a0 + t)] == s->L.ci[size_t(l0 + t)];
    if (ok) {
      pre[size_t(r)] = cnt + 1;
      ++s->prefix_rows;
      s->prefix_entries += cnt + 1;
    }
  }
  if (s->prefix_rows == 0) return;
  s->apre.resize(s->order.size());
  s->pqrng = s->qrng;
  for (size_t q = 0; q < s->order.size(); ++q) {
    const int32_t id = s->order[q];
    s->apre[q] = -1;
    if (id < n) {
      if (id < lim && pre[size_t(id)] > 0) s->apre[q] = s->A.rp[id];
    } else if (id - n < lim && pre[size_t(id - n)] > 0) {
      s->pqrng[2 * q] = -(s->A.rp[id - n] + pre[size_t(id - n)]) - 1;
    }
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
      const int64_t slot = std::min<int64_t>(int64_t(s->ready[r]) + std::max(0, s->spmv_delay), last);
      key[n + r] = int32_t(2 * slot + 1);
      cost[n + r] = std::max(1, s->A.rp[r + 1] - s->A.rp[r]);
    }
    counting_order(key, 2 * (last + 1), s->order);
    cut_runs(s->order, key, cost, s->rows_per_item, s->max_item_nnz, s->item_ptr, s->spmv_item_scale);
    s->trsv_items.clear();
    s->spmv_items.clear();
    for (size_t t = 0; t + 1 < s->item_ptr.size(); ++t) {
      if (s->order[s->item_ptr[t]] < n) s->trsv_items.push_back(int32_t(t));
      else s->spmv_items.push_back(int32_t(t));
    }
    // One hop per joint wavefront, one step inside each.
    s->est_level_us = double(s->joint_depth) * (kEstHop + kEstStep);
    s->corder.clear();
    s->citem_ptr.clear();
    s->ctrsv_items.clear();
    s->clloc.clear();
    s->celoc.clear();
    s->chunk_chain = 0;
    s->max_local_depth = 0;
    s->est_chunk_us = 0.0;
    const bool try_chunks = s->coarsen >= 2 || (s->coarsen == 0 && mesh_like(n, s->L.rp, s->L.ci, 0, 1, s->level));
    s->cqrng.clear();
    if (try_chunks && n > 0) build_chunks(s);
    position_ranges(s, s->order, s->qrng);
    prefix_ranges(s);
    if (!s->corder.empty()) position_ranges(s, s->corder, s->cqrng);
    s->chunked = !s->ctrsv_items.empty() &&
                 (s->coarsen == 2 || s->coarsen == 3 || s->est_chunk_us < 0.8 * s->est_level_us);
    // regions: on request, or by default on a mesh-like DAG where the
    // region model beats the coarsened plan's pipelined estimate clearly
    s->rorder.clear();
    s->regioned = false;
    s->est_region_us = 0.0;
    if (n > 0 && (s->coarsen == 3 || (s->coarsen == 0 && try_chunks && !s->ctrsv_items.empty()))) {
      // regions of region_rows rows, halved while the largest one's LDS
      // does not fit a wavefront's share
      size_t lds = 0;
      for (int32_t R = s->region_rows;; R /= 2) {
        build_regions(s, R);
        lds = region_lds_bytes(s->region_rows_max, s->region_entries_max, s->region_ext_max,
                               s->region_batches_max, 8);
        if (lds <= kRegionLdsMax || R <= 64) break;
      }
      position_ranges(s, s->rorder, s->rqrng);
      s->regioned = lds <= kRegionLdsMax && (s->coarsen == 3 || s->est_region_us < 0.85 * s->est_chunk_pipe_us);
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
    // one batch of 64 / lanes rows per item: the rows of a batch run side by
    // side, batches of one item would run one after the other
    const int32_t per_batch = std::max(1, 64 / std::max(1, s->lanes_trsv));
    cut_runs(s->order, key, cost, std::min(s->rows_per_item, per_batch), s->max_item_nnz, s->item_ptr);
    s->trsv_items.clear();
    for (size_t t = 0; t + 1 < s->item_ptr.size(); ++t) s->trsv_items.push_back(int32_t(t));
    if (s->kind == SF_IC0_TRSV) {
      position_ranges(s, s->order, s->qrng);
      s->prng.resize(2 * s->order.size());
      for (size_t q = 0; q < s->order.size(); ++q) {
        const int32_t i = s->order[q];
        s->prng[2 * q] = s->pair_ptr[size_t(s->L.rp[i])];
        s->prng[2 * q + 1] = s->pair_ptr[size_t(s->L.rp[i + 1] - 1)];
      }
    } else {
      s->qrng.clear();
      s->prng.clear();
    }
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
    s->est_back_level_us = double(s->back_depth) * (kEstHop + kEstStep);
    s->bcorder.clear();
    s->bcitem_ptr.clear();
    s->bclloc.clear();
    s->bceloc.clear();
    s->back_chunk_chain = 0;
    s->est_back_chunk_us = 0.0;
    const bool try_back = s->coarsen == 2 || s->coarsen == 3 ||
                          (s->coarsen == 0 && mesh_like(n, s->LT.rp, s->LT.ci, 1, 0, s->rlevel));
    s->est_back_chunk_pipe_us = 0.0;
    if (try_back && n > 0) build_back_chunks(s);
    s->bchunked = !s->bcitem_ptr.empty() &&
                  (s->coarsen == 2 || s->coarsen == 3 || s->est_back_chunk_us < 0.8 * s->est_back_level_us);
    // backward regions, as the forward ones: on request, or on a mesh-like
    // DAG where their estimate beats the coarsened plan's clearly
    s->bregioned = false;
    s->brorder.clear();
    s->est_back_region_us = 0.0;
    if (n > 0 && (s->coarsen == 3 || (s->coarsen == 0 && try_back && !s->bcitem_ptr.empty()))) {
      size_t lds = 0;
      for (int32_t R = std::min(s->region_rows, 1024);; R /= 2) {
        build_back_regions(s, R);
        lds = region_lds_bytes(s->back_region_rows_max, s->back_region_entries_max, s->back_region_ext_max,
                               s->back_region_batches_max, 8);
        if (lds <= kRegionLdsMax || R <= 64) break;
      }
      s->bregioned = lds <= kRegionLdsMax &&
                     (s->coarsen == 3 || s->est_back_region_us < 0.85 * s->est_back_chunk_pipe_us);
    }
  }
}

static void build_pairs(sf_schedule_s* s) {
  const Pattern& L = s->L;
  const int64_t nnz = L.nnz();
  s->pair_ptr.assign(size_t(nnz) + 1, 0);
  s->pair_u.clear();
  s->pair_q.clear();
  s->piv.assign(size_t(nnz), -1);
  for (int32_t i = 0; i < L.nrows; ++i) {
    const int32_t r0 = L.rp[i], rd = L.rp[i + 1] - 1;
    for (int32_t p = r0; p < rd; ++p) {
      const int32_t j = L.ci[p];
      s->piv[size_t(p)] = L.rp[j + 1] - 1;  // the pivot L_jj closes row j
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
  // a sentinel past the last list: a list's end position is always a valid
  // index, so the executor's index loads need no bounds branch
  s->pair_u.push_back(-1);
  s->pair_q.push_back(0);
}

// SpILU0 intersection lists, one list per stored entry (i, j) of A: pairs
// (t << 16 | u, q) for every stored k = column of entry u of row i with
// k < min(i, j) and (k, j) stored at position q of row k (u_kj).  Lists of
// a row's entries are contiguous, in entry order.
static void build_pairs_ilu(sf_schedule_s* s) {
  const Pattern& A = s->L;
  const int64_t nnz = A.nnz();
  s->pair_ptr.assign(size_t(nnz) + 1, 0);
  s->pair_u.clear();
  s->pair_q.clear();
  for (int32_t i = 0; i < A.nrows; ++i) {
    const int32_t r0 = A.rp[i], r1 = A.rp[i + 1];
    for (int32_t p = r0; p < r1; ++p) {
      const int32_t j = A.ci[p];
      const int32_t lim = std::min(i, j);
      for (int32_t pk = r0; pk < r1 && A.ci[pk] < lim; ++pk) {
        const int32_t k = A.ci[pk];
        // (k, j) in row k: binary search over its sorted columns
        const int32_t* b = A.ci.data() + A.rp[k];
        const int32_t* e = A.ci.data() + A.rp[k + 1];
        const int32_t* f = std::lower_bound(b, e, j);
        if (f != e && *f == j) {
          s->pair_u.push_back(((p - r0) << 16) | (pk - r0));
          s->pair_q.push_back(int32_t(f - A.ci.data()));
        }
      }
      s->pair_ptr[size_t(p) + 1] = int32_t(s->pair_u.size());
    }
  }
  s->pair_u.push_back(-1);  // sentinel, as for SpIC0
  s->pair_q.push_back(0);
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

  // SpILU0: the position of each row's diagonal (the pattern is the whole
  // of A; the entries left of it are the row's dependences).
  if (s->kind == SF_ILU0_TRSV) {
    s->dpos.assign(size_t(n), 0);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1]; ++p)
        if (s->L.ci[p] == i) s->dpos[size_t(i)] = p;
  }
  // end of row i's dependences: its diagonal
  auto dep_end = [&](int64_t i) { return s->kind == SF_ILU0_TRSV ? s->dpos[size_t(i)] : s->L.rp[i + 1] - 1; };

  // Levels (wavefront numbers) of the SpTRSV (SpIC0, SpILU0) DAG.
  s->level.assign(size_t(n), 0);
  int32_t depth = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t lv = 0;
    for (int32_t p = s->L.rp[i]; p < dep_end(i); ++p) lv = std::max(lv, s->level[s->L.ci[p]] + 1);
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
    if (s->kind == SF_ILU0_TRSV) {
      // Table 2, combination 6: 2 size_A / max(size_A, size_L + 2n), size_L the
      // stored entries left of the diagonal
      double sl = 0.0;
      for (int64_t i = 0; i < n; ++i) sl += double(s->dpos[size_t(i)] - s->L.rp[i]);
      s->reuse = nl > 0 ? 2.0 * nl / std::max(nl, sl + 2.0 * double(n)) : 0.0;
      build_pairs_ilu(s);
    } else {
      s->reuse = nl > 0 ? 2.0 * nl / std::max(nl, nl + 2.0 * double(n)) : 0.0;
      build_pairs(s);
    }
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
  if (s->kind == SF_IC0_TRSV || s->kind == SF_ILU0_TRSV) {
    // one lane per stored entry of an SpIC0 / SpILU0 row
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
  s->coarsen = o.coarsen;
  cut_items(s);
  return SF_OK;
}

// Check a forward plan against every DAG edge: each iteration appears once,
// and every edge u -> v has item(u) < item(v), or (coarsened plans) u and v
// share an item with u on an earlier local wavefront.
static int validate_plan(const sf_schedule_s* s, const std::vector<int32_t>& order,
                         const std::vector<int32_t>& item_ptr, const std::vector<uint8_t>* lloc) {
  const int64_t n = s->n, m = s->m;
  const int64_t N = s->kind == SF_TRSV_SPMV ? n + m : n;
  std::vector<int32_t> item(size_t(N), -1), pos(size_t(N), -1);
  const int64_t nitems = int64_t(item_ptr.size()) - 1;
  if (item_ptr.empty() || item_ptr[0] != 0 || item_ptr.back() != N) return 1;
  for (int64_t t = 0; t < nitems; ++t) {
    if (item_ptr[t + 1] <= item_ptr[t]) return 2;
    for (int32_t q = item_ptr[t]; q < item_ptr[t + 1]; ++q) {
      const int32_t u = order[q];
      if (u < 0 || u >= N || item[u] >= 0) return 3;
      item[u] = int32_t(t);
      pos[u] = q;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1] - 1; ++p) {
      const int32_t j = s->L.ci[p];
      if (item[j] < item[i]) continue;
      if (lloc && item[j] == item[i] && (*lloc)[pos[j]] < (*lloc)[pos[i]] &&
          s->celoc[size_t(p)] == uint8_t(pos[j] - item_ptr[item[i]]))
        continue;
      return 4;
    }
  if (s->kind == SF_TRSV_SPMV)
    for (int64_t r = 0; r < m; ++r)
      for (int32_t p = s->A.rp[r]; p < s->A.rp[r + 1]; ++p)
        if (!(item[s->A.ci[p]] < item[n + r])) return 5;
  if (lloc) {
    // item-local rows sorted by local wavefront; entries outside the item flagged external
    for (int64_t t = 0; t < nitems; ++t)
      for (int32_t q = item_ptr[t] + 1; q < item_ptr[t + 1]; ++q)
        if ((*lloc)[q] < (*lloc)[q - 1]) return 6;
    for (int64_t i = 0; i < n; ++i)
      for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1] - 1; ++p)
        if (s->celoc[size_t(p)] != 0xFF && item[s->L.ci[p]] != item[i]) return 7;
  }
  return 0;
}

// The backward plan: every edge lambda_j -> lambda_i (L_ji stored, j > i)
// has item(j) < item(i), or (coarsened) the same item with j on an earlier
// local wavefront and the entry's slot naming j.
static int validate_back_plan(const sf_schedule_s* s, const std::vector<int32_t>& order,
                              const std::vector<int32_t>& item_ptr, const std::vector<uint8_t>* lloc) {
  const int64_t n = s->n;
  std::vector<int32_t> item(size_t(n), -1), pos(size_t(n), -1);
  if (item_ptr.empty() || item_ptr[0] != 0 || item_ptr.back() != n) return 11;
  for (size_t t = 0; t + 1 < item_ptr.size(); ++t) {
    if (item_ptr[t + 1] <= item_ptr[t]) return 12;
    for (int32_t q = item_ptr[t]; q < item_ptr[t + 1]; ++q) {
      const int32_t u = order[q];
      if (u < 0 || u >= n || item[u] >= 0) return 13;
      item[u] = int32_t(t);
      pos[u] = q;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = s->LT.rp[i] + 1; p < s->LT.rp[i + 1]; ++p) {
      const int32_t j = s->LT.ci[p];
      if (item[j] < item[i]) {
        if (lloc && s->bceloc[size_t(p)] != 0xFF) return 15;
        continue;
      }
      if (lloc && item[j] == item[i] && (*lloc)[pos[j]] < (*lloc)[pos[i]] &&
          s->bceloc[size_t(p)] == uint8_t(pos[j] - item_ptr[item[i]]))
        continue;
      return 14;
    }
  return 0;
}

// SpILU0 plans: each row once, and every dependence k -> i (a stored (i, k),
// k < i) goes to a later item.
static int validate_ilu_plan(const sf_schedule_s* s) {
  const int64_t n = s->n;
  std::vector<int32_t> item(size_t(n), -1);
  if (s->item_ptr.empty() || s->item_ptr[0] != 0 || s->item_ptr.back() != n) return 21;
  for (size_t t = 0; t + 1 < s->item_ptr.size(); ++t) {
    if (s->item_ptr[t + 1] <= s->item_ptr[t]) return 22;
    for (int32_t q = s->item_ptr[t]; q < s->item_ptr[t + 1]; ++q) {
      const int32_t u = s->order[q];
      if (u < 0 || u >= n || item[u] >= 0) return 23;
      item[u] = int32_t(t);
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = s->L.rp[i]; p < s->dpos[size_t(i)]; ++p)
      if (!(item[s->L.ci[p]] < item[i])) return 24;
  return 0;
}

// The region plan: every iteration once, edges between regions go forward,
// edges inside a region to a later local wavefront through its in-region
// code; each batch is level-pure, at most 64 rows, and the batches tile the
// region; every external code names the column in the region's list, and a
// batch uses no external input first used by a later batch.
static int validate_region_plan(const sf_schedule_s* s) {
  const int64_t n = s->n, m = s->m;
  int r = validate_plan(s, s->rorder, s->ritem_ptr, nullptr);
  if (r == 4) {  // in-region edges are checked below
    r = 0;
  }
  if (r != 0) return r;
  const int64_t N = n + m;
  const int64_t nitems = int64_t(s->ritem_ptr.size()) - 1;
  std::vector<int32_t> item(size_t(N), -1), pos(size_t(N), -1), batch_of(s->rorder.size(), -1);
  for (int64_t t = 0; t < nitems; ++t)
    for (int32_t q = s->ritem_ptr[t]; q < s->ritem_ptr[t + 1]; ++q) {
      item[s->rorder[q]] = int32_t(t);
      pos[s->rorder[q]] = q;
    }
  if (int64_t(s->rbatch_ptr.size()) != nitems + 1 || int64_t(s->rext_ptr.size()) != nitems + 1) return 10;
  for (int64_t t = 0; t < nitems; ++t) {
    const int32_t q0 = s->ritem_ptr[t], q1 = s->ritem_ptr[t + 1];
    const int32_t b0 = s->rbatch_ptr[t], b1 = s->rbatch_ptr[t + 1];
    if (b1 == b0) continue;  // SpMV item
    if (q1 - q0 > 32767 || s->rext_ptr[t + 1] - s->rext_ptr[t] > 32767) return 11;
    if (s->rbatch[2 * b0] != q0) return 12;
    int32_t ovf = 0;  // overflow offsets: the entries past kRegionAhead of the earlier rows
    for (int32_t q = q0; q < q1; ++q) {
      const int32_t i = s->rorder[q];
      if (i >= n || s->rroff[q] != ovf) return 20;
      ovf += std::max(0, s->L.rp[i + 1] - 1 - s->L.rp[i] - kRegionAhead);
    }
    if (ovf > s->region_entries_max) return 20;
    for (int32_t b = b0; b < b1; ++b) {
      const int32_t pb = s->rbatch[2 * b], pe = b + 1 < b1 ? s->rbatch[2 * (b + 1)] : q1;
      if (pe <= pb || pe - pb > 64) return 13;
      for (int32_t q = pb; q < pe; ++q) {
        if (s->rorder[q] >= n || s->rlloc[q] != s->rlloc[pb]) return 14;
        batch_of[q] = b - b0;
      }
      if (b + 1 < b1 && (s->rlloc[pe] < s->rlloc[pb] || s->rbatch[2 * (b + 1) + 1] < s->rbatch[2 * b + 1])) return 15;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    const int32_t t = item[i];
    const int32_t b0 = s->rbatch_ptr[t];
    for (int32_t p = s->L.rp[i]; p < s->L.rp[i + 1] - 1; ++p) {
      const int32_t j = s->L.ci[p];
      const int code = s->rcode[size_t(p)];
      if (item[j] == t) {
        if (code & 0x8000 || code != pos[j] - s->ritem_ptr[t] || !(s->rlloc[pos[j]] < s->rlloc[pos[i]])) return 16;
      } else {
        const int xi = code & 0x7fff;
        if (!(code & 0x8000) || !(item[j] < t) || xi >= s->rext_ptr[t + 1] - s->rext_ptr[t]) return 17;
        if (s->rext[size_t(s->rext_ptr[t] + xi)] != j) return 18;
        if (xi >= (batch_of[pos[i]] + 1 < s->rbatch_ptr[t + 1] - b0 ? s->rbatch[2 * (b0 + batch_of[pos[i]] + 1) + 1]
                                                                     : s->rext_ptr[t + 1] - s->rext_ptr[t]))
          return 19;  // used before its first-use batch
      }
    }
  }
  for (int64_t r2 = 0; r2 < m; ++r2)
    for (int32_t p = s->A.rp[r2]; p < s->A.rp[r2 + 1]; ++p)
      if (!(item[s->A.ci[p]] < item[n + r2])) return 5;
  return 0;
}

// The backward region plan: every row once, batches of one local level and
// at most 64 rows, overflow offsets, and for every transposed-solve edge
// (L_ji stored, j > i) either an in-region code naming j's slot at an
// earlier local level or an external input of the region listed under j,
// with j's region claimed earlier.
static int validate_back_region_plan(const sf_schedule_s* s) {
  const int64_t n = s->n;
  if (int64_t(s->brorder.size()) != n) return 30;
  const int64_t nitems = int64_t(s->britem_ptr.size()) - 1;
  if (int64_t(s->brbatch_ptr.size()) != nitems + 1 || int64_t(s->brext_ptr.size()) != nitems + 1) return 31;
  std::vector<int32_t> item(size_t(n), -1), pos(size_t(n), -1);
  for (int64_t t = 0; t < nitems; ++t)
    for (int32_t q = s->britem_ptr[t]; q < s->britem_ptr[t + 1]; ++q) {
      const int32_t i = s->brorder[q];
      if (i < 0 || i >= n || item[i] >= 0) return 32;
      item[i] = int32_t(t);
      pos[i] = q;
    }
  for (int64_t t = 0; t < nitems; ++t) {
    const int32_t q0 = s->britem_ptr[t], q1 = s->britem_ptr[t + 1];
    const int32_t b0 = s->brbatch_ptr[t], b1 = s->brbatch_ptr[t + 1];
    if (b1 <= b0 || s->brbatch[2 * b0] != q0) return 33;
    for (int32_t b = b0; b < b1; ++b) {
      const int32_t pb = s->brbatch[2 * b], pe = b + 1 < b1 ? s->brbatch[2 * (b + 1)] : q1;
      if (pe <= pb || pe - pb > 64) return 34;
      for (int32_t q = pb; q < pe; ++q)
        if (s->brlloc[q] != s->brlloc[pb]) return 34;
      if (b + 1 < b1 && s->brlloc[pe] < s->brlloc[pb]) return 34;
    }
    int32_t ovf = 0;
    for (int32_t q = q0; q < q1; ++q) {
      const int32_t i = s->brorder[q];
      if (s->brroff[q] != ovf) return 35;
      ovf += std::max(0, s->LT.rp[i + 1] - 1 - s->LT.rp[i] - kRegionAhead);
    }
    if (ovf > s->back_region_entries_max || q1 - q0 > s->back_region_rows_max) return 35;
  }
  for (int64_t i = 0; i < n; ++i) {
    const int32_t t = item[i];
    for (int32_t p = s->LT.rp[i] + 1; p < s->LT.rp[i + 1]; ++p) {
      const int32_t j = s->LT.ci[p];
      const int code = s->brcode[size_t(p)];
      if (j <= i) return 36;
      if (item[j] == t) {
        if ((code & 0x8000) || code != pos[j] - s->britem_ptr[t] || !(s->brlloc[pos[j]] < s->brlloc[pos[i]]))
          return 37;
      } else {
        const int xi = code & 0x7fff;
        if (!(code & 0x8000) || !(item[j] < t) || xi >= s->brext_ptr[t + 1] - s->brext_ptr[t]) return 38;
        if (s->brext[size_t(s->brext_ptr[t] + xi)] != j) return 38;
      }
    }
  }
  return 0;
}

int validate_forward(const sf_schedule_s* s) {
  if (s->kind == SF_ILU0_TRSV) return validate_ilu_plan(s);
  int r = validate_plan(s, s->order, s->item_ptr, nullptr);
  if (r == 0 && s->chunked) r = validate_plan(s, s->corder, s->citem_ptr, &s->clloc);
  if (r == 0 && s->regioned) r = validate_region_plan(s);
  if (r == 0 && s->has_back) r = validate_back_plan(s, s->border, s->bitem_ptr, nullptr);
  if (r == 0 && s->bchunked) r = validate_back_plan(s, s->bcorder, s->bcitem_ptr, &s->bclloc);
  if (r == 0 && s->bregioned) r = validate_back_region_plan(s);
  return r;
}

}  // namespace sf
