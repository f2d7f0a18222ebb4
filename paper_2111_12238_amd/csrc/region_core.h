// The region executor's core (k_region.hip, k_bwd.hip): a region's rows
// staged into LDS, a polling wavefront storing the region's external inputs
// into LDS as they are published, and a computing wavefront running the
// region's local wavefronts in batches of up to 64 rows (one row per lane),
// every input read from LDS.  Each row folds its terms in ascending column
// order and divides by its diagonal: the sequential substitution's
// arithmetic, so results are bit-identical to it.  Every file that includes
// this header must keep multiply-add contraction off.
#pragma once

#include "ts_items.h"

namespace sf {
namespace {

using dev::is_pending;
using dev::ld_co;
using dev::publishable;
using dev::st_co;

constexpr int kRegionThreads = 128;  // a computing and a polling wavefront

// Per row of a region, in LDS: the first kRegionAhead entries' values and
// input slots (past the row's end: value 0 and the slot holding 0), the
// right-hand side, the diagonal, the iteration id and the row's overflow
// entries (offset and count).  One record is read in one round of
// independent LDS loads.
template <typename T>
struct alignas(16) RowHead {
  T v[kRegionAhead];
  T b, d;
  uint16_t s[kRegionAhead];
  int32_t id;
  uint16_t oo, on;
};
static_assert(sizeof(RowHead<double>) == 64 && sizeof(RowHead<float>) == 48, "region row record");

// The region's LDS, carved from the dynamic allocation (sizes: the largest
// region's rows R, overflow entries O, external inputs X and batches NB;
// region_lds_bytes): row records [R]; x slots [R + X + 1] -- the region's
// rows, its external inputs (slot R + k for input k), a slot holding 0;
// overflow values [O]; external columns [X]; batch table [NB + 1];
// overflow slots [O].
template <typename T>
struct RegionLds {
  RowHead<T>* head;
  T *xa, *ov;
  int32_t *xc, *bt;
  uint16_t* oc;
  int zero;  // the slot holding 0
};

template <typename T>
__device__ __forceinline__ RegionLds<T> carve(char* base, int R, int O, int X, int NB) {
  RegionLds<T> L;
  L.head = reinterpret_cast<RowHead<T>*>(base);
  L.xa = reinterpret_cast<T*>(L.head + R);
  L.zero = R + X;
  L.ov = L.xa + R + X + 1;
  L.xc = reinterpret_cast<int32_t*>(L.ov + O);
  L.bt = L.xc + X;
  L.oc = reinterpret_cast<uint16_t*>(L.bt + NB + 1);
  return L;
}

template <typename T>
__device__ __forceinline__ T pending_value() {
  return __builtin_bit_cast(T, dev::Pending<T>::bits);
}

template <typename T>
__device__ __forceinline__ T lds_get(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <typename T>
__device__ __forceinline__ void lds_put(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// An input read from LDS and, while still pending (an external input the
// poller has not stored yet), read again.
template <typename T>
__device__ __forceinline__ T wait_slot(const T* xa, int slot, T v) {
  while (is_pending(v)) {
    __builtin_amdgcn_s_sleep(1);
    v = lds_get(xa + slot);
  }
  return v;
}

// One region (item `item`, claim positions [q0, q1), batches [b0, b1)) on a
// block of two wavefronts.  Both stage the region into LDS; then wavefront
// 1 polls the region's inputs from other regions in order of first use
// (its first W lanes own inputs lane, lane + W, ..., one load each in
// flight, storing each into LDS once published) while wavefront 0 runs the
// batches, reading every input from LDS and waiting there for the ones not
// yet stored.  The computing wavefront thus issues no global load after the
// staging, its batches never wait for its own stores, and the row records
// of the next batch are read while the current one computes, so a batch's
// dependent chain is one LDS read of its inputs, its terms and its division.
// Row k of a region into its LDS record: id, right-hand side b, diagonal
// d and the off-diagonal entries (value, code -- in-region position, or
// 0x8000 | external index) in the definition's column order, the first
// kRegionAhead in the record, the rest at overflow offset oo.
template <typename T>
__device__ __forceinline__ void stage_row(const RegionLds<T>& L, int R, int k, int id, T b, T d, int oo, int cnt,
                                          const T* vals, const int32_t* vmap, int p0, const uint16_t* code) {
  RowHead<T> h;
#pragma unroll
  for (int u = 0; u < kRegionAhead; ++u) {
    h.v[u] = T(0);
    h.s[u] = uint16_t(L.zero);
  }
  // four entries at a time, their loads issued together
  for (int u0 = 0; u0 < cnt; u0 += 4) {
    int pm[4], cd[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int p = p0 + min(u0 + e, cnt - 1);
      pm[e] = vmap ? vmap[p] : p;
      cd[e] = code[p];
    }
    T v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = dev::ld_stream(vals + pm[e]);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = u0 + e;
      if (u >= cnt) break;
      const uint16_t slot = uint16_t((cd[e] & 0x8000) ? R + (cd[e] & 0x7fff) : cd[e]);
      if (u < kRegionAhead) {
        h.v[u] = v[e];
        h.s[u] = slot;
      } else {
        L.ov[oo + u - kRegionAhead] = v[e];
        L.oc[oo + u - kRegionAhead] = slot;
      }
    }
  }
  h.b = b;
  h.d = d;
  h.id = id;
  h.oo = uint16_t(oo);
  h.on = uint16_t(cnt > kRegionAhead ? cnt - kRegionAhead : 0);
  L.head[k] = h;
}

// One region (item `item`, claim positions [q0, q1), batches [b0, b1)) on a
// block of two wavefronts; X is the solution (published through the
// readiness protocol), stage(L, k) stages row k (stage_row).
template <typename T, typename Stage>
__device__ void region_core(const RegionArgs& r, int item, int q0, int q1, int b0, int b1, char* lds,
                            unsigned long long* tr, T* X, const LaunchState& ls, unsigned long long* rtrace,
                            const Stage& stage) {
  const int R = r.rows_max;
  const RegionLds<T> L = carve<T>(lds, R, r.entries_max, r.ext_max, r.batches_max);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nr = q1 - q0;
  const int x0 = r.ext_ptr[item];
  const int nx = r.ext_ptr[item + 1] - x0;
  for (int k = tid; k < nr; k += kRegionThreads) stage(L, k);
  for (int k = tid; k < nx; k += kRegionThreads) {
    L.xc[k] = r.ext[x0 + k];
    L.xa[R + k] = pending_value<T>();
  }
  for (int k = tid; k < b1 - b0; k += kRegionThreads) L.bt[k] = r.batch[2 * (b0 + k)] - q0;
  if (tid == 0) {
    L.bt[b1 - b0] = nr;
    L.xa[L.zero] = T(0);
  }
  __syncthreads();
  if (tr && tid == 0) tr[1] = __builtin_amdgcn_s_memrealtime();  // staged
  if (wid == 1) {
    // the poller: lane l watches input k_lo + l, where k_lo is the first
    // input (in first-use order) not yet stored; each round the window
    // slides past its stored prefix, so every lane moves on to a pending
    // input at once.  At most r.poll_lanes lanes read per round, and until
    // the region's first input is stored (a region claimed ahead of its
    // producers waits there) only r.poll_gate: every read is one more
    // request on the memory side, where the publications travel too.  After
    // a round in which nothing became final it backs off r.poll_sleep.
    uint64_t done = 0;  // bit l: input k_lo + l stored
    int k_lo = 0;
    int32_t spins = 0;
    while (k_lo < nx) {
      const int k = k_lo + lane;
      const int F = k_lo == 0 ? r.poll_gate : r.poll_lanes;
      const bool want = lane < F && k < nx && !((done >> lane) & 1ull);
      T v = pending_value<T>();
      if (want) v = ld_co(X + L.xc[k]);
      const bool got = want && !is_pending(v);
      if (got) lds_put(L.xa + R + k, v);
      const uint64_t g = __ballot(got);
      if (tr && k_lo == 0 && g != 0 && lane == 0) tr[5] = __builtin_amdgcn_s_memrealtime();  // first input
      done |= g;
      const int sh = done == ~0ull ? 64 : __builtin_ctzll(~done);
      k_lo += sh;
      done = sh == 64 ? 0ull : done >> sh;
      if (!dev::all_poll_round(spins, ls)) {
        // watchdog: release every input still pending so the region drains
        for (int q = lane; q < nx; q += 64) lds_put(L.xa + R + q, T(0));
        break;
      }
      if (g == 0)
        for (int z = 0; z < r.poll_sleep; ++z) __builtin_amdgcn_s_sleep(2);
    }
    if (tr && lane == 0) tr[2] = __builtin_amdgcn_s_memrealtime();  // every input observed
    return;
  }
  // the computing wavefront: one batch (<= 64 rows of one local wavefront,
  // consecutive slots) at a time, each lane one row.  The batch table is
  // held one window of 64 entries at a time, one per lane (batches win ..
  // win + 61 of a window need entries up to win + 63); within a window the
  // next batch's records are read unconditionally (the last batch reads its
  // own again), so no load waits on a branch.
  const int nb = b1 - b0;
  for (int win = 0; win < nb; win += 62) {
    const int btw = L.bt[min(win + lane, nb)];
    const int wend = min(nb, win + 62);
    int pb = __builtin_amdgcn_readlane(btw, 0);
    int pe = __builtin_amdgcn_readlane(btw, 1);
    bool mine = lane < pe - pb;
    RowHead<T> h = L.head[mine ? pb + lane : pb];
    for (int bl = win; bl < wend; ++bl) {
      const RowHead<T> c = h;
      const bool cmine = mine;
      const int ck = pb + lane;
      T xx[kRegionAhead];
#pragma unroll
      for (int u = 0; u < kRegionAhead; ++u) xx[u] = lds_get(L.xa + c.s[u]);
      const int bn = min(bl + 1, nb - 1) - win;
      pb = __builtin_amdgcn_readlane(btw, bn);
      pe = __builtin_amdgcn_readlane(btw, bn + 1);
      mine = lane < pe - pb;
      h = L.head[mine ? pb + lane : pb];
      bool wait = false;
#pragma unroll
      for (int u = 0; u < kRegionAhead; ++u) wait |= is_pending(xx[u]);
      if (wait) {
#pragma unroll
        for (int u = 0; u < kRegionAhead; ++u) xx[u] = wait_slot(L.xa, c.s[u], xx[u]);
      }
      T acc = c.b;
#pragma unroll
      for (int u = 0; u < kRegionAhead; ++u) acc = acc - c.v[u] * xx[u];
      // entries past the first kRegionAhead, in order
      for (int t = c.oo; t < c.oo + c.on; ++t) {
        const int slot = L.oc[t];
        acc = acc - L.ov[t] * wait_slot(L.xa, slot, lds_get(L.xa + slot));
      }
      const T xk = publishable(acc / c.d);
      if (cmine) {
        lds_put(L.xa + ck, xk);
        if (rtrace) dev::stamp_publish(rtrace, true, c.id);
        st_co(X + c.id, xk);
      }
      if (tr && bl == 0 && lane == 0) tr[6] = __builtin_amdgcn_s_memrealtime();  // first batch published
      __builtin_amdgcn_wave_barrier();
    }
  }
}

}  // namespace
}  // namespace sf
