// Static two-level plans of the SpTRSV -> SpMV pair, for the measured
// comparison of the paper's own schedule with the dynamic executor.
//
// MSP (Sec. 3.2, Algorithm 1), for G1 = the SpTRSV DAG (the kernel with
// dependences, hence the head DAG) and G2 = the SpMV rows (no edges, tail
// DAG, forward pairing):
//  (i)   vertex partitioning: consecutive wavefronts of G1 are grouped into
//        s-partitions and each s-partition's connected components into at
//        most r w-partitions balanced by cost (the role the paper gives to
//        its LBC partitioner); forward pairing: the SpMV rows whose every
//        input lies in one w-partition H form its self-contained pair T,
//        placed as a w-partition of the next s-partition; the other rows
//        (inputs in several w-partitions) form a partition U placed after
//        the s-partition of their last input;
//  (ii)  slack numbers SN(v) = P - l(v) - height(v) on the joint DAG; pairs
//        whose partitions both have slack 0 are merged (T runs after H in
//        H's w-partition); SpMV rows with positive slack are taken out and
//        dispersed: each w-partition lighter than its s-partition's
//        heaviest by more than eps = 0.001 |V| takes rows of its own pair
//        first, then any slack row whose window includes this s-partition;
//        rows whose window ends here are divided evenly over up to r
//        w-partitions of it (opening new ones when it has fewer);
//  (iii) separated packing (the pair's reuse ratio is below one, Table 2):
//        a w-partition runs its SpTRSV rows by wavefront, then its SpMV
//        rows in row order.
// The fused wavefront baseline (Sec. 4): one s-partition per wavefront of
// the joint DAG, its SpTRSV and SpMV rows in w-partitions of up to 64 rows.
//
// The vertex cost is the paper's c(v): the nonzeros a row touches.
#include <algorithm>
#include <cstdint>
#include <functional>
#include <numeric>
#include <queue>
#include <vector>

#include "schedule.h"

namespace sf {
namespace {

constexpr int kBatchRows = 64;  // rows per executor batch (one wavefront of 64 lanes)

// Union-find with union by size, component costs at the roots and an undo
// log (no path compression), so a tentatively added wavefront can be taken
// back out of a window.
struct UndoDSU {
  std::vector<int32_t> parent, size;
  std::vector<int64_t> cost;
  std::vector<int32_t> log;  // roots that were attached, most recent last
  explicit UndoDSU(size_t n) : parent(n), size(n, 1), cost(n, 0) { std::iota(parent.begin(), parent.end(), 0); }
  int32_t find(int32_t x) const {
    while (parent[size_t(x)] != x) x = parent[size_t(x)];
    return x;
  }
  bool unite(int32_t a, int32_t b) {
    a = find(a);
    b = find(b);
    if (a == b) return false;
    if (size[size_t(a)] < size[size_t(b)]) std::swap(a, b);
    parent[size_t(b)] = a;
    size[size_t(a)] += size[size_t(b)];
    cost[size_t(a)] += cost[size_t(b)];
    log.push_back(b);
    return true;
  }
  void undo_to(size_t mark) {
    while (log.size() > mark) {
      const int32_t b = log.back();
      log.pop_back();
      const int32_t a = parent[size_t(b)];
      size[size_t(a)] -= size[size_t(b)];
      cost[size_t(a)] -= cost[size_t(b)];
      parent[size_t(b)] = b;
    }
  }
};

struct Part {
  std::vector<int32_t> rows;  // iteration ids (SpTRSV i, SpMV n + r)
  int64_t cost = 0;
  int32_t pair_of = -1;       // for a pair partition T: its H partition
  int32_t sn = 0;             // partition slack number
};

void finish(sf_schedule_s* s, StaticPlan& P, const std::vector<std::vector<int32_t>>& sparts,
            const std::vector<Part>& parts) {
  const int64_t n = s->n;
  P.s_ptr.assign(1, 0);
  P.w_ptr.assign(1, 0);
  P.order.clear();
  P.w_batch.assign(1, 0);
  P.batch_ptr.assign(1, 0);
  for (const auto& sp : sparts) {
    int32_t nw = 0;
    for (int32_t w : sp) {
      const Part& pt = parts[size_t(w)];
      if (pt.rows.empty()) continue;
      // batches: runs of one kind and, for SpTRSV rows, one wavefront
      const size_t q0 = P.order.size();
      for (size_t k = 0; k < pt.rows.size(); ++k) {
        const int32_t v = pt.rows[k];
        const size_t q = P.order.size();
        bool cut = q == q0 || q - size_t(P.batch_ptr.back()) >= size_t(kBatchRows);
        if (!cut) {
          const int32_t u = P.order.back();
          cut = (u < n) != (v < n) || (v < n && s->level[size_t(u)] != s->level[size_t(v)]);
        }
        if (cut && q != q0) P.batch_ptr.push_back(int32_t(q));
        P.order.push_back(v);
      }
      P.batch_ptr.push_back(int32_t(P.order.size()));
      P.w_ptr.push_back(int32_t(P.order.size()));
      P.w_batch.push_back(int32_t(P.batch_ptr.size()) - 1);
      ++nw;
    }
    if (nw > 0) P.s_ptr.push_back(P.s_ptr.back() + nw);
  }
  P.qrng.resize(2 * P.order.size());
  for (size_t q = 0; q < P.order.size(); ++q) {
    const int32_t id = P.order[q];
    if (id < n) {
      P.qrng[2 * q] = s->L.rp[size_t(id)];
      P.qrng[2 * q + 1] = s->L.rp[size_t(id) + 1] - 1;
    } else {
      P.qrng[2 * q] = s->A.rp[size_t(id - n)];
      P.qrng[2 * q + 1] = s->A.rp[size_t(id - n) + 1];
    }
  }
  P.built = true;
}

int64_t trsv_cost(const sf_schedule_s* s, int32_t i) { return s->L.rp[size_t(i) + 1] - s->L.rp[size_t(i)]; }
int64_t spmv_cost(const sf_schedule_s* s, int32_t r) {
  return std::max<int64_t>(1, s->A.rp[size_t(r) + 1] - s->A.rp[size_t(r)]);
}

void build_wavefront(sf_schedule_s* s, StaticPlan& P) {
  const int64_t n = s->n, m = s->m;
  const int32_t D = std::max(s->joint_depth, s->depth);
  std::vector<std::vector<int32_t>> trsv_at(size_t(D) + 1), spmv_at(size_t(D) + 1);
  for (int64_t i = 0; i < n; ++i) trsv_at[size_t(s->level[size_t(i)])].push_back(int32_t(i));
  for (int64_t r = 0; r < m; ++r) spmv_at[size_t(s->ready[size_t(r)])].push_back(int32_t(n + r));
  std::vector<Part> parts;
  std::vector<std::vector<int32_t>> sparts;
  for (size_t l = 0; l < trsv_at.size(); ++l) {
    std::vector<int32_t> ws;
    for (const auto* rows : {&trsv_at[l], &spmv_at[l]})
      for (size_t b = 0; b < rows->size(); b += kBatchRows) {
        Part pt;
        pt.rows.assign(rows->begin() + long(b), rows->begin() + long(std::min(rows->size(), b + kBatchRows)));
        ws.push_back(int32_t(parts.size()));
        parts.push_back(std::move(pt));
      }
    if (!ws.empty()) sparts.push_back(std::move(ws));
  }
  finish(s, P, sparts, parts);
}

void build_msp(sf_schedule_s* s, StaticPlan& P, int r) {
  const int64_t n = s->n, m = s->m;
  const int32_t DL = s->depth;
  const auto& lrp = s->L.rp;
  const auto& lci = s->L.ci;
  const auto& arp = s->A.rp;
  const auto& aci = s->A.ci;
  // rows of G1 by wavefront
  std::vector<int32_t> lptr(static_cast<size_t>(DL) + 1, 0), lrows(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) ++lptr[size_t(s->level[size_t(i)]) + 1];
  for (size_t l = 1; l < lptr.size(); ++l) lptr[l] += lptr[l - 1];
  {
    std::vector<int32_t> at(lptr.begin(), lptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) lrows[size_t(at[size_t(s->level[size_t(i)])]++)] = int32_t(i);
  }
  // (i) vertex partitioning: grow a window of wavefronts while it keeps at
  // least min(r, independent pieces on either side) connected components
  // and can still be split into that many w-partitions of balanced cost
  // (its largest component at most twice their mean cost)
  UndoDSU dsu(size_t(std::max<int64_t>(n, 1)));
  for (int64_t i = 0; i < n; ++i) dsu.cost[size_t(i)] = trsv_cost(s, int32_t(i));
  std::vector<Part> parts;
  std::vector<std::vector<int32_t>> sparts;       // H partitions of each window, then T / U appended
  std::vector<int32_t> window_of_level(size_t(DL) + 1, 0);
  std::vector<int32_t> wpart(size_t(n), -1), spart(size_t(n), -1);
  int32_t lb = 0;
  while (lb < DL) {
    int64_t comps = lptr[size_t(lb) + 1] - lptr[size_t(lb)];  // one wavefront: no edges inside it
    int64_t total = 0, biggest = 0;
    for (int32_t q = lptr[size_t(lb)]; q < lptr[size_t(lb) + 1]; ++q) {
      const int64_t c = dsu.cost[size_t(lrows[size_t(q)])];
      total += c;
      biggest = std::max(biggest, c);
    }
    int32_t ub = lb + 1;
    while (ub < DL) {
      const size_t mark = dsu.log.size();
      const int64_t width = lptr[size_t(ub) + 1] - lptr[size_t(ub)];
      int64_t merged_comps = comps + width, merged_total = total, merged_big = biggest;
      for (int32_t q = lptr[size_t(ub)]; q < lptr[size_t(ub) + 1]; ++q) {
        const int32_t i = lrows[size_t(q)];
        merged_total += dsu.cost[size_t(i)];
        for (int32_t p = lrp[size_t(i)]; p < lrp[size_t(i) + 1] - 1; ++p)
          if (s->level[size_t(lci[size_t(p)])] >= lb && dsu.unite(lci[size_t(p)], i)) --merged_comps;
        merged_big = std::max(merged_big, dsu.cost[size_t(dsu.find(i))]);
      }
      const int64_t bins = std::min<int64_t>(r, std::max(comps, width));
      if (merged_comps >= bins && merged_big * std::min<int64_t>(r, merged_comps) <= 2 * merged_total) {
        comps = merged_comps;
        total = merged_total;
        biggest = merged_big;
        ++ub;
      } else {
        dsu.undo_to(mark);
        break;
      }
    }
    // components of the window -> at most r w-partitions (largest first, to the lightest bin)
    const int32_t sidx = int32_t(sparts.size());
    std::vector<int32_t> root_id;
    std::vector<int64_t> comp_cost;
    std::vector<std::vector<int32_t>> comp_rows;
    {
      std::vector<std::pair<int32_t, int32_t>> rr;  // (root, row)
      for (int32_t q = lptr[size_t(lb)]; q < lptr[size_t(ub)]; ++q) {
        const int32_t i = lrows[size_t(q)];
        rr.emplace_back(dsu.find(i), i);
      }
      std::sort(rr.begin(), rr.end());
      for (size_t k = 0; k < rr.size(); ++k) {
        if (k == 0 || rr[k].first != rr[k - 1].first) {
          comp_rows.emplace_back();
          comp_cost.push_back(0);
        }
        comp_rows.back().push_back(rr[k].second);
        comp_cost.back() += trsv_cost(s, rr[k].second);
      }
    }
    const size_t nbins = std::min<size_t>(size_t(std::max(r, 1)), comp_rows.size());
    std::vector<int32_t> cidx(comp_rows.size());
    std::iota(cidx.begin(), cidx.end(), 0);
    std::stable_sort(cidx.begin(), cidx.end(), [&](int32_t a, int32_t b) { return comp_cost[size_t(a)] > comp_cost[size_t(b)]; });
    std::vector<int32_t> ws(nbins);
    using Bin = std::pair<int64_t, int32_t>;  // (cost, bin)
    std::priority_queue<Bin, std::vector<Bin>, std::greater<Bin>> heap;
    for (size_t b = 0; b < nbins; ++b) {
      ws[b] = int32_t(parts.size());
      parts.emplace_back();
      heap.emplace(0, int32_t(b));
    }
    for (int32_t c : cidx) {
      Bin b = heap.top();
      heap.pop();
      Part& pt = parts[size_t(ws[size_t(b.second)])];
      pt.rows.insert(pt.rows.end(), comp_rows[size_t(c)].begin(), comp_rows[size_t(c)].end());
      pt.cost += comp_cost[size_t(c)];
      heap.emplace(pt.cost, b.second);
    }
    for (int32_t w : ws) {
      Part& pt = parts[size_t(w)];
      std::sort(pt.rows.begin(), pt.rows.end(), [&](int32_t a, int32_t b) {
        return s->level[size_t(a)] != s->level[size_t(b)] ? s->level[size_t(a)] < s->level[size_t(b)] : a < b;
      });
      for (int32_t i : pt.rows) {
        wpart[size_t(i)] = w;
        spart[size_t(i)] = sidx;
      }
    }
    for (int32_t l = lb; l < ub; ++l) window_of_level[size_t(l)] = sidx;
    sparts.push_back(ws);
    dsu.log.clear();  // the window is final; its unions stay (later windows never join it)
    lb = ub;
  }
  const int32_t nb = int32_t(sparts.size());  // windows; s-partition nb holds what follows the last
  sparts.emplace_back();
  window_of_level[size_t(DL)] = nb;
  P.parts = r;
  // forward pairing: SpMV rows with every input in one w-partition H form
  // H's pair T (next s-partition); the others join U of the w-partition
  // holding their last input (after its s-partition)
  std::vector<int32_t> pair_part(parts.size(), -1), unc_part(parts.size(), -1);
  std::vector<int32_t> home(size_t(m), -1);   // partition of each SpMV row
  std::vector<int32_t> earliest(size_t(m), 0);
  std::vector<int32_t> free_rows;             // SpMV rows without inputs
  for (int64_t rr = 0; rr < m; ++rr) {
    const int32_t p0 = arp[size_t(rr)], p1 = arp[size_t(rr) + 1];
    if (p0 == p1) {
      free_rows.push_back(int32_t(rr));
      continue;
    }
    // the w-partition of the first input, and the input with the latest
    // s-partition (then the largest w-partition id)
    const int32_t w0 = wpart[size_t(aci[size_t(p0)])];
    int32_t last_w = w0, last_s = spart[size_t(aci[size_t(p0)])];
    bool contained = true;
    for (int32_t p = p0; p < p1; ++p) {
      const int32_t j = aci[size_t(p)];
      const int32_t wj = wpart[size_t(j)], sj = spart[size_t(j)];
      contained = contained && wj == w0;
      if (sj > last_s || (sj == last_s && wj > last_w)) {
        last_s = sj;
        last_w = wj;
      }
    }
    const int32_t owner = contained ? w0 : last_w;
    int32_t& slot = contained ? pair_part[size_t(owner)] : unc_part[size_t(owner)];
    if (slot < 0) {
      slot = int32_t(parts.size());
      parts.emplace_back();
      parts.back().pair_of = contained ? owner : -1;
      sparts[size_t(last_s) + 1].push_back(slot);
    }
    parts[size_t(slot)].rows.push_back(int32_t(n + rr));
    parts[size_t(slot)].cost += spmv_cost(s, int32_t(rr));
    home[size_t(rr)] = slot;
    earliest[size_t(rr)] = last_s + 1;
  }
  // (ii) slack numbers on the joint DAG: heights from the sinks, in reverse
  // row order (an SpTRSV row's successors have larger ids)
  const int32_t D = std::max<int32_t>(s->joint_depth, DL);
  std::vector<int32_t> height(size_t(n), 0);
  for (int64_t rr = 0; rr < m; ++rr)
    for (int32_t p = arp[size_t(rr)]; p < arp[size_t(rr) + 1]; ++p) height[size_t(aci[size_t(p)])] = 1;
  for (int64_t i = n - 1; i >= 0; --i)
    for (int32_t p = lrp[size_t(i)]; p < lrp[size_t(i) + 1] - 1; ++p) {
      int32_t& h = height[size_t(lci[size_t(p)])];
      h = std::max(h, height[size_t(i)] + 1);
    }
  auto sn_trsv = [&](int32_t i) { return D - 1 - s->level[size_t(i)] - height[size_t(i)]; };
  auto sn_spmv = [&](int32_t rr) { return D - 1 - s->ready[size_t(rr)]; };
  for (Part& pt : parts) {
    int32_t sn = INT32_MAX;
    for (int32_t v : pt.rows) sn = std::min(sn, v < n ? sn_trsv(v) : sn_spmv(int32_t(v - n)));
    pt.sn = pt.rows.empty() ? 0 : std::max(sn, 0);
  }
  // merging: a pair (H, T) with slack 0 on both sides runs in H's w-partition
  int32_t merged = 0;
  for (size_t t = 0; t < parts.size(); ++t) {
    Part& T = parts[t];
    if (T.pair_of < 0 || T.rows.empty()) continue;
    Part& H = parts[size_t(T.pair_of)];
    if (H.sn == 0 && T.sn == 0) {
      H.rows.insert(H.rows.end(), T.rows.begin(), T.rows.end());
      H.cost += T.cost;
      for (int32_t v : T.rows) home[size_t(v - n)] = T.pair_of;
      T.rows.clear();
      T.cost = 0;
      ++merged;
    }
  }
  // slack rows leave their partitions: SpMV rows with SN > 0 still in a T or U
  struct Slack {
    int32_t row, earliest, latest, pair;
  };
  std::vector<Slack> slack;
  std::vector<uint8_t> is_slack(size_t(m), 0);
  for (int64_t rr = 0; rr < m; ++rr) {
    const int32_t h = home[size_t(rr)];
    const bool in_h = h >= 0 && parts[size_t(h)].pair_of < 0 && !parts[size_t(h)].rows.empty() &&
                      parts[size_t(h)].rows.front() < n;  // merged into its H
    if (h < 0 || in_h) continue;
    if (sn_spmv(int32_t(rr)) <= 0) continue;
    const int32_t lat_level = std::min<int32_t>(s->ready[size_t(rr)] + sn_spmv(int32_t(rr)), DL);
    const int32_t latest = std::max(earliest[size_t(rr)], window_of_level[size_t(lat_level)]);
    slack.push_back({int32_t(rr), earliest[size_t(rr)], latest, parts[size_t(h)].pair_of});
    is_slack[size_t(rr)] = 1;
  }
  for (int32_t rr : free_rows) slack.push_back({rr, 0, nb, -1});
  for (Part& pt : parts) {
    if (pt.rows.empty() || pt.rows.front() < n) continue;
    std::vector<int32_t> keep;
    pt.cost = 0;
    for (int32_t v : pt.rows)
      if (!is_slack[size_t(v - n)]) {
        keep.push_back(v);
        pt.cost += spmv_cost(s, int32_t(v - n));
      }
    pt.rows.swap(keep);
  }
  // slacked vertex assignment, s-partition by s-partition
  std::vector<std::vector<int32_t>> pair_slack(parts.size());
  std::vector<int32_t> by_earliest(slack.size());
  std::iota(by_earliest.begin(), by_earliest.end(), 0);
  std::stable_sort(by_earliest.begin(), by_earliest.end(),
                   [&](int32_t a, int32_t b) { return slack[size_t(a)].earliest < slack[size_t(b)].earliest; });
  for (size_t k = 0; k < slack.size(); ++k)
    if (slack[k].pair >= 0) pair_slack[size_t(slack[k].pair)].push_back(int32_t(k));
  std::vector<uint8_t> placed(slack.size(), 0);
  using Urg = std::pair<int32_t, int32_t>;  // (latest, slack index)
  std::priority_queue<Urg, std::vector<Urg>, std::greater<Urg>> pool;
  size_t next_in = 0;
  const int64_t eps = std::max<int64_t>(1, (n + m) / 1000);
  int32_t moved = 0;
  std::vector<int64_t> due_at(size_t(nb) + 1, 0);  // unplaced slack rows by last s-partition
  int64_t unplaced = int64_t(slack.size());
  for (const Slack& sl : slack) ++due_at[size_t(sl.latest)];
  auto place = [&](int32_t w, int32_t k) {
    Part& pt = parts[size_t(w)];
    pt.rows.push_back(int32_t(n + slack[size_t(k)].row));
    pt.cost += spmv_cost(s, slack[size_t(k)].row);
    placed[size_t(k)] = 1;
    --due_at[size_t(slack[size_t(k)].latest)];
    --unplaced;
    ++moved;
  };
  for (int32_t i = 0; i <= nb; ++i) {
    while (next_in < by_earliest.size() && slack[size_t(by_earliest[next_in])].earliest <= i) {
      const int32_t k = by_earliest[next_in++];
      pool.emplace(slack[size_t(k)].latest, k);
    }
    std::vector<int32_t> ws;
    for (int32_t w : sparts[size_t(i)])
      if (!parts[size_t(w)].rows.empty()) ws.push_back(w);
    int64_t top = 0;
    for (int32_t w : ws) top = std::max(top, parts[size_t(w)].cost);
    for (int32_t w : ws) {
      Part& pt = parts[size_t(w)];
      // rows of its own pair first: they run after it in the same w-partition
      for (int32_t k : pair_slack[size_t(w)]) {
        if (top - pt.cost <= eps) break;
        if (!placed[size_t(k)]) place(w, k);
      }
      while (top - pt.cost > eps && !pool.empty()) {
        const int32_t k = pool.top().second;
        pool.pop();
        if (!placed[size_t(k)]) place(w, k);
      }
    }
    // rows whose window ends here are divided evenly over up to r
    // w-partitions of this s-partition (new ones are opened when it has
    // fewer, at most one per executor batch of rows)
    const size_t due = size_t(i == nb ? unplaced : due_at[size_t(i)]);
    const size_t want = std::min<size_t>(size_t(std::max(r, 1)), (due + kBatchRows - 1) / kBatchRows);
    while (ws.size() < want) {
      ws.push_back(int32_t(parts.size()));
      sparts[size_t(i)].push_back(ws.back());
      parts.emplace_back();
    }
    using Bin = std::pair<int64_t, int32_t>;
    std::priority_queue<Bin, std::vector<Bin>, std::greater<Bin>> light;
    for (int32_t w : ws) light.emplace(parts[size_t(w)].cost, w);
    while (!pool.empty() && (pool.top().first <= i || i == nb)) {
      const int32_t k = pool.top().second;
      pool.pop();
      if (placed[size_t(k)]) continue;
      Bin b = light.top();
      light.pop();
      place(b.second, k);
      light.emplace(parts[size_t(b.second)].cost, b.second);
    }
  }
  // anything still out (its window had no w-partition) runs in a last s-partition
  {
    Part tail;
    for (size_t k = 0; k < slack.size(); ++k)
      if (!placed[k]) {
        tail.rows.push_back(int32_t(n + slack[k].row));
        placed[k] = 1;
      }
    if (!tail.rows.empty()) {
      sparts.emplace_back(1, int32_t(parts.size()));
      parts.push_back(std::move(tail));
    }
  }
  // (iii) separated packing: SpTRSV rows by wavefront, then SpMV rows by row
  for (Part& pt : parts)
    std::stable_sort(pt.rows.begin(), pt.rows.end(), [&](int32_t a, int32_t b) {
      const bool ta = a < n, tb = b < n;
      if (ta != tb) return ta;
      if (ta && s->level[size_t(a)] != s->level[size_t(b)]) return s->level[size_t(a)] < s->level[size_t(b)];
      return a < b;
    });
  P.merged = merged;
  P.slack_moved = moved;
  finish(s, P, sparts, parts);
}

}  // namespace

StaticPlan& static_plan(sf_schedule_s* s, int plan) { return plan == 0 ? s->msp : s->wavefront; }

sf_status build_static(sf_schedule_s* s, int plan) {
  if (s->kind != SF_TRSV_SPMV || (plan != 0 && plan != 1)) return SF_ERR_ARG;
  StaticPlan& P = static_plan(s, plan);
  if (P.built && (plan == 1 || P.parts == s->msp_parts)) return SF_OK;
  try {
    if (plan == 0) build_msp(s, P, s->msp_parts);
    else build_wavefront(s, P);
  } catch (const std::bad_alloc&) {
    return SF_ERR_OOM;
  }
  return SF_OK;
}

}  // namespace sf
