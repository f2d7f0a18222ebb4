// Row-sum building block shared by the forward and adjoint executors.
//
// A work item holds up to 64 independent rows; row slot s (lane s) owns the
// CSR range [r0, r0 + len).  stream_accumulate computes, for every row slot,
//     acc_s  (-|+)=  val[p] * vec[col[p]]   for p = r0 .. r0 + len - 1
// one rounded product at a time in ascending p, which is exactly the
// sequential definition's arithmetic.  The entries of all rows are
// concatenated and dealt to the 64 lanes, kRounds per lane, so one round of
// independent loads fetches every index, value and vec element of the item;
// products go through LDS and each row's lane folds its own.  vec may be
// read through the value-as-flag readiness protocol (dev_common.h).
// Every file that includes this header must keep multiply-add contraction
// off so the products are rounded as written.
#pragma once

#include "dev_common.h"

namespace sf {
namespace dev {

constexpr int kRounds = 8;           // entries per lane per pass
constexpr int kPass = 64 * kRounds;  // entries per pass of one wavefront
constexpr int kWaves = kBlockThreads / 64;
static_assert(kPass >= kChunkEntries, "a coarsened item must fit one stream pass");

template <typename T>
struct WaveLds {
  int32_t pos[kPass];  // CSR position of each stream entry of the current pass
  T prod[kPass];       // rounded products of the current pass
};

// Wait until every vec[j[e]] of the wavefront (j[e] < 0: unused slot) is
// published, updating xv.  Two ways to wait, chosen per round by how many
// lanes still wait (ALL_BELOW):
//  - every lane re-reads all its pending entries (up to ALL_BELOW waiting
//    lanes): the last value is seen within one round trip of its
//    publication, at one request per pending entry and round;
//  - one lane polls: among the pending entries the wavefront watches the
//    one with the largest index -- producers are claimed in topological
//    order, so it is usually the last to be published -- and once it is,
//    every lane re-reads its still-pending entries; the election repeats if
//    any remain.  One request per round keeps the traffic of many waiting
//    wavefronts low, at about a third of a round trip more latency.
// ALL_BELOW = 64 always takes the first way (latency-bound schedules: one
// item waits on a few producers); 0 always the second.
// One round of "every lane re-reads its pending entries"; false once the
// watchdog has fired (the caller then drains).
__device__ __forceinline__ bool all_poll_round(int32_t& spins, const LaunchState& ls) {
  if (++spins >= ls.spin_limit) {
    report_timeout(ls);
    return false;
  }
  return (spins & 63) != 0 || !timed_out(ls);
}

template <typename T, int R, int ALL_BELOW = 32>
__device__ __forceinline__ void wait_ready(const T* vec, const int (&j)[R], T (&xv)[R], int lane,
                                           const LaunchState& ls) {
  int32_t spins = 0;
  for (;;) {
    int jmax = -1;
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (j[e] >= 0 && is_pending(xv[e])) jmax = max(jmax, j[e]);
    const unsigned long long mask = __ballot(jmax >= 0);
    if (mask == 0) return;
    if (ALL_BELOW >= 64 || __popcll(mask) <= ALL_BELOW) {
#pragma unroll
      for (int e = 0; e < R; ++e)
        if (j[e] >= 0 && is_pending(xv[e])) xv[e] = ld_co(vec + j[e]);
      if (!all_poll_round(spins, ls)) return;
      continue;
    }
    int wmax = jmax;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wmax = max(wmax, __shfl_xor(wmax, d, 64));
    const int leader = __ffsll(static_cast<long long>(__ballot(jmax == wmax))) - 1;
    if (lane == leader) {
      const T got = poll_value(vec + wmax, ls);
#pragma unroll
      for (int e = 0; e < R; ++e)
        if (j[e] == wmax) xv[e] = got;
    }
    if (timed_out(ls)) return;  // watchdog fired in this launch: drain
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (j[e] >= 0 && is_pending(xv[e])) xv[e] = ld_co(vec + j[e]);
  }
}

// As wait_ready, for values at arbitrary addresses p[e] (nullptr: unused
// slot), e.g. factor entries.  The watched value is the pending one at the
// highest address.
template <typename T, int R, int ALL_BELOW = 32>
__device__ __forceinline__ void wait_ptrs(const T* (&p)[R], T (&v)[R], int lane, const LaunchState& ls) {
  int32_t spins = 0;
  for (;;) {
    unsigned long long best = 0;
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (p[e] && is_pending(v[e])) best = max(best, (unsigned long long)p[e]);
    const unsigned long long mask = __ballot(best != 0);
    if (mask == 0) return;
    if (ALL_BELOW >= 64 || __popcll(mask) <= ALL_BELOW) {
#pragma unroll
      for (int e = 0; e < R; ++e)
        if (p[e] && is_pending(v[e])) v[e] = ld_co(p[e]);
      if (!all_poll_round(spins, ls)) return;
      continue;
    }
    unsigned long long wbest = best;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
      wbest = max(wbest, (unsigned long long)__shfl_xor((long long)wbest, d, 64));
    const int leader = __ffsll(static_cast<long long>(__ballot(best == wbest))) - 1;
    if (lane == leader) {
      const T* w = reinterpret_cast<const T*>(wbest);
      const T got = poll_value(w, ls);
#pragma unroll
      for (int e = 0; e < R; ++e)
        if (p[e] == w) v[e] = got;
    }
    if (timed_out(ls)) return;  // watchdog fired in this launch: drain
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (p[e] && is_pending(v[e])) v[e] = ld_co(p[e]);
  }
}

// VEC: 0 = vec final and read through the caches, 1 = vec final but written
// in this launch by another kernel phase (device-coherent read), 2 = vec
// produced concurrently (device-coherent read + readiness protocol), 3 = vec
// produced concurrently, first read through the caches and re-read
// device-coherently while pending.  A cached read returns either the value
// or the pending pattern (a value changes once per launch, from pending to
// final, and every launch starts with the caches invalidated), so 3 is as
// exact as 2 and lets neighbouring gathers share cache lines.
// MAPPED: the value of entry p is val[map[p]] (a transposed view).
// trace: optional per-item timestamp slots (see the trace mode of k_ts.hip).
// Returns the row slot's accumulator (meaningful on lanes < nr).
template <typename T, bool SUB, int VEC, bool MAPPED>
__device__ __forceinline__ T stream_accumulate(int nr, int r0, int len, T acc, const int32_t* __restrict__ col,
                                               const int32_t* __restrict__ map, const T* __restrict__ val,
                                               const T* vec, int lane, WaveLds<T>& w, const LaunchState& ls,
                                               unsigned long long* trace = nullptr) {
  const bool mine = lane < nr;
  if (!mine) len = 0;
  // exclusive prefix sum of the row lengths over the item's row slots
  int incl = len;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int off = incl - len;
  const int total = __shfl(incl, 63, 64);
  for (int base = 0; base < total; base += kPass) {
    // each row's lane lays its entries' CSR positions into this pass's window
    if (mine) {
      const int lo = max(off, base), hi = min(off + len, base + kPass);
      for (int t = lo; t < hi; ++t) w.pos[t - base] = r0 + (t - off);
    }
    __builtin_amdgcn_wave_barrier();
    int j[kRounds];
    T v[kRounds], xv[kRounds];
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      j[e] = -1;
      v[e] = T(0);
      if (k < total) {
        const int p = w.pos[k - base];
        j[e] = ld_stream(col + p);
        v[e] = MAPPED ? val[ld_stream(map + p)] : ld_stream(val + p);
      }
    }
#pragma unroll
    for (int e = 0; e < kRounds; ++e)
      xv[e] = j[e] >= 0 ? ((VEC == 0 || VEC == 3) ? vec[j[e]] : ld_co(vec + j[e])) : T(0);
    if (trace && lane == 0) trace[1] = __builtin_amdgcn_s_memrealtime();  // loads issued
    if constexpr (VEC >= 2) wait_ready<T, kRounds>(vec, j, xv, lane, ls);
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      if (k < total) w.prod[k - base] = v[e] * xv[e];
    }
    if (trace && lane == 0) trace[2] = __builtin_amdgcn_s_memrealtime();  // inputs ready
    __builtin_amdgcn_wave_barrier();
    if (mine) {
      // ascending order, one rounding per term; LDS reads issued 8 ahead
      const int lo = max(off, base) - base;
      const int hi = min(off + len, base + kPass) - base;
      int t = lo;
      for (; t + 8 <= hi; t += 8) {
        T pr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pr[u] = w.prod[t + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = SUB ? acc - pr[u] : acc + pr[u];
      }
      for (; t < hi; ++t) acc = SUB ? acc - w.prod[t] : acc + w.prod[t];
    }
    __builtin_amdgcn_wave_barrier();
  }
  return acc;
}

// ---- prefix fusion (level items) ----
//
// SpTRSV row i also folds SpMV row i's prefix -- its entries up to the
// diagonal, whose columns are exactly L's row i off-diagonals -- from the x
// values the row gathers anyway: y_i's partial sum, in A's entry order
// from 0.  apos holds each stream entry's A position (-1: the row has no
// prefix) and prod2 the prefix products.
template <typename T>
struct WaveLdsPre : WaveLds<T> {
  int32_t apos[kPass];
  T prod2[kPass];
};

// stream_accumulate for SpTRSV rows (SUB) with a prefix: as above, and for
// rows with a0 >= 0 (the A position of the row's first prefix entry) also
// acc2 += A[a0 + t] * vec[col] in entry order t (acc2 from 0).
template <typename T, int VEC>
__device__ __forceinline__ T stream_accumulate_pre(int nr, int r0, int len, int a0, T acc, T& acc2,
                                                   const int32_t* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ aval, const T* vec, int lane,
                                                   WaveLdsPre<T>& w, const LaunchState& ls,
                                                   unsigned long long* trace = nullptr) {
  const bool mine = lane < nr;
  if (!mine) len = 0;
  int incl = len;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int off = incl - len;
  const int total = __shfl(incl, 63, 64);
  acc2 = T(0);
  for (int base = 0; base < total; base += kPass) {
    if (mine) {
      const int lo = max(off, base), hi = min(off + len, base + kPass);
      for (int t = lo; t < hi; ++t) {
        w.pos[t - base] = r0 + (t - off);
        w.apos[t - base] = a0 >= 0 ? a0 + (t - off) : -1;
      }
    }
    __builtin_amdgcn_wave_barrier();
    int j[kRounds];
    T v[kRounds], av[kRounds], xv[kRounds];
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      j[e] = -1;
      v[e] = T(0);
      av[e] = T(0);
      if (k < total) {
        const int p = w.pos[k - base];
        const int q = w.apos[k - base];
        j[e] = ld_stream(col + p);
        v[e] = ld_stream(val + p);
        if (q >= 0) av[e] = ld_stream(aval + q);
      }
    }
#pragma unroll
    for (int e = 0; e < kRounds; ++e)
      xv[e] = j[e] >= 0 ? ((VEC == 0 || VEC == 3) ? vec[j[e]] : ld_co(vec + j[e])) : T(0);
    if (trace && lane == 0) trace[1] = __builtin_amdgcn_s_memrealtime();
    if constexpr (VEC >= 2) wait_ready<T, kRounds>(vec, j, xv, lane, ls);
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      if (k < total) {
        w.prod[k - base] = v[e] * xv[e];
        w.prod2[k - base] = av[e] * xv[e];
      }
    }
    if (trace && lane == 0) trace[2] = __builtin_amdgcn_s_memrealtime();
    __builtin_amdgcn_wave_barrier();
    if (mine) {
      const int lo = max(off, base) - base;
      const int hi = min(off + len, base + kPass) - base;
      int t = lo;
      for (; t + 8 <= hi; t += 8) {
        T pr[8], pq[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          pr[u] = w.prod[t + u];
          pq[u] = w.prod2[t + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          acc = acc - pr[u];
          acc2 = acc2 + pq[u];
        }
      }
      for (; t < hi; ++t) {
        acc = acc - w.prod[t];
        acc2 = acc2 + w.prod2[t];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  return acc;
}

// stream_accumulate for SpMV rows whose prefix was folded by their SpTRSV
// row: the row's lane starts from y0 (its partial sum, published by the
// SpTRSV row's item through the readiness protocol, read here device-
// coherently and waited for with the entries' x) instead of 0; y0 == nullptr
// for a row without a prefix.
template <typename T, int VEC>
__device__ __forceinline__ T stream_accumulate_from(int nr, int r0, int len, const T* y0,
                                                    const int32_t* __restrict__ col, const T* __restrict__ val,
                                                    const T* vec, int lane, WaveLds<T>& w, const LaunchState& ls,
                                                    unsigned long long* trace = nullptr) {
  const bool mine = lane < nr;
  if (!mine) len = 0;
  T acc = (mine && y0) ? ld_co(y0) : T(0);  // in flight with the first pass
  bool first = true;
  int incl = len;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int off = incl - len;
  const int total = __shfl(incl, 63, 64);
  for (int base = 0; base == 0 || base < total; base += kPass) {
    if (mine) {
      const int lo = max(off, base), hi = min(off + len, base + kPass);
      for (int t = lo; t < hi; ++t) w.pos[t - base] = r0 + (t - off);
    }
    __builtin_amdgcn_wave_barrier();
    int j[kRounds];
    T v[kRounds], xv[kRounds];
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      j[e] = -1;
      v[e] = T(0);
      if (k < total) {
        const int p = w.pos[k - base];
        j[e] = ld_stream(col + p);
        v[e] = ld_stream(val + p);
      }
    }
#pragma unroll
    for (int e = 0; e < kRounds; ++e)
      xv[e] = j[e] >= 0 ? ((VEC == 0 || VEC == 3) ? vec[j[e]] : ld_co(vec + j[e])) : T(0);
    if (trace && lane == 0) trace[1] = __builtin_amdgcn_s_memrealtime();  // loads issued
    if constexpr (VEC >= 2) wait_ready<T, kRounds>(vec, j, xv, lane, ls);
    if (first) {
      // the partial sum: re-read while pending (all lanes poll together)
      int32_t spins = 0;
      while (__ballot(mine && y0 && is_pending(acc)) != 0) {
        if (mine && y0 && is_pending(acc)) acc = ld_co(y0);
        if (!all_poll_round(spins, ls)) break;
      }
      first = false;
    }
    if (trace && lane == 0) trace[2] = __builtin_amdgcn_s_memrealtime();  // inputs ready
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      if (k < total) w.prod[k - base] = v[e] * xv[e];
    }
    __builtin_amdgcn_wave_barrier();
    if (mine) {
      const int lo = max(off, base) - base;
      const int hi = min(off + len, base + kPass) - base;
      int t = lo;
      for (; t + 8 <= hi; t += 8) {
        T pr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) pr[u] = w.prod[t + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = acc + pr[u];
      }
      for (; t < hi; ++t) acc = acc + w.prod[t];
    }
    __builtin_amdgcn_wave_barrier();
  }
  return acc;
}

// ---- coarsened items: rows on several local wavefronts ----
//
// Local wavefront steps.  The owner lane keeps its row's first NT terms in
// registers: a factor pv (the rounded product for an entry outside the
// item, the matrix value for an item-local column, 0 for an unused slot)
// and the LDS slot of the value it multiplies (xl[64] holds 1.0 for the
// first and last kind), so a step is NT LDS reads, NT products and NT
// subtractions with no selects; multiplying by 1.0 and subtracting +0.0 are
// exact, so the terms and their order are still the definition's.
template <typename T, int NT>
__device__ __forceinline__ T chunk_steps(WaveLds<T>& w, T* xl, T* vec, bool mine, int myloc, int maxloc, int off,
                                         int len, int row, int lane, T acc, T dii, unsigned long long* rtr) {
  constexpr int kOne = 64;
  T pv[NT];
  int pq[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    pv[u] = T(0);
    pq[u] = kOne;
    if (u < len) {
      const int q = w.pos[off + u];
      pv[u] = w.prod[off + u];
      pq[u] = q == 0xFF ? kOne : q;
    }
  }
  T mine_x = T(0);
  for (int s = 0; s <= maxloc; ++s) {
    if (mine && myloc == s) {
      T xq[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) xq[u] = xl[pq[u]];
#pragma unroll
      for (int u = 0; u < NT; ++u) acc = acc - pv[u] * xq[u];
      for (int t = off + NT; t < off + len; ++t) {
        const int q = w.pos[t];
        acc = acc - (q == 0xFF ? w.prod[t] : w.prod[t] * xl[q]);
      }
      const T x = publishable(acc / dii);
      xl[lane] = x;
      if (rtr) stamp_publish(rtr, true, row);
      st_co(vec + row, x);
      mine_x = x;
    }
    __builtin_amdgcn_wave_barrier();
  }
  return mine_x;
}

// Solve the rows of a coarsened item.  Row slot s (lane s < nr) owns the
// entries [r0, r0 + len) of (col, val) -- val[map[p]] when MAPPED -- and
// eloc[p] is the slot of the entry's column inside the item, or 0xFF.  All
// the item's entries are dealt to the lanes in one pass (the inspector keeps
// an item's entries within one pass): an item-local entry loads nothing
// more; the others load vec[col] through the readiness protocol, waited for
// together.  Then the local wavefronts run in order (chunk_steps): each row
// folds its entries in ascending position -- a product taken from LDS, or
// the value times the item's own result kept in LDS -- divides by dii,
// keeps the result for the later wavefronts and publishes it in vec[row].
// Every product is rounded once and every row folds in ascending order, as
// in the sequential substitution.  Returns the lane's own result.  xl holds
// 65 values: 64 slots and the constant 1.0 at [64].
template <typename T, bool MAPPED>
__device__ __forceinline__ T chunk_solve(int nr, int r0, int len, int myloc, int maxloc, T acc, T dii,
                                         const int32_t* __restrict__ col, const int32_t* __restrict__ map,
                                         const T* __restrict__ val, const uint8_t* __restrict__ eloc, T* vec,
                                         int row, int lane, WaveLds<T>& w, T* xl, const LaunchState& ls,
                                         unsigned long long* tr, unsigned long long* rtr = nullptr) {
  const bool mine = lane < nr;
  if (!mine) len = 0;
  int incl = len;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int off = incl - len;
  const int total = __shfl(incl, 63, 64);
  if (mine)
    for (int t = off; t < off + len; ++t) w.pos[t] = r0 + (t - off);
  __builtin_amdgcn_wave_barrier();
  int j[kRounds], sl[kRounds];
  T v[kRounds], xv[kRounds];
#pragma unroll
  for (int e = 0; e < kRounds; ++e) {
    const int k = lane + 64 * e;
    j[e] = -1;
    sl[e] = 0xFF;
    v[e] = T(0);
    if (k < total) {
      const int p = w.pos[k];
      sl[e] = int(ld_stream(eloc + p));
      v[e] = MAPPED ? val[ld_stream(map + p)] : ld_stream(val + p);
      if (sl[e] == 0xFF) j[e] = ld_stream(col + p);
    }
  }
#pragma unroll
  for (int e = 0; e < kRounds; ++e) xv[e] = j[e] >= 0 ? ld_co(vec + j[e]) : T(0);
  if (tr && lane == 0) tr[1] = __builtin_amdgcn_s_memrealtime();
  wait_ready<T, kRounds, 64>(vec, j, xv, lane, ls);  // few producers, latency-bound
  // LDS: prod[k] = rounded product (outside entry) or the value (local entry);
  // pos[k] = slot of the local column, or 0xFF
#pragma unroll
  for (int e = 0; e < kRounds; ++e) {
    const int k = lane + 64 * e;
    if (k < total) {
      w.prod[k] = sl[e] == 0xFF ? v[e] * xv[e] : v[e];
      w.pos[k] = sl[e];
    }
  }
  if (tr && lane == 0) tr[2] = __builtin_amdgcn_s_memrealtime();
  __builtin_amdgcn_wave_barrier();
  int maxlen = len;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, d, 64));
  if (maxlen <= 4) return chunk_steps<T, 4>(w, xl, vec, mine, myloc, maxloc, off, len, row, lane, acc, dii, rtr);
  return chunk_steps<T, 8>(w, xl, vec, mine, myloc, maxloc, off, len, row, lane, acc, dii, rtr);
}

}  // namespace dev
}  // namespace sf
