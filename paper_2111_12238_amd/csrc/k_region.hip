// Fused SpTRSV -> SpMV executor on the region plan (gfx950).
//
// A region is a set of up to a few hundred SpTRSV rows grown around a seed
// (inspect.cpp, build_regions), run by a block of two wavefronts: the
// region's row data (right-hand sides, diagonals, the values and in-region
// codes of the off-diagonals) are staged into LDS when it is claimed; then
// one wavefront runs its local wavefronts in order, in batches of up to 64
// rows (one row per lane), while the other polls the region's inputs from
// other regions (published through the readiness protocol) and stores each
// into LDS as soon as it is final.  A row's in-region inputs come from the
// region's x in LDS and its other inputs from that LDS copy, waited for by
// that row only, so a region starts as soon as its first rows' inputs
// exist and runs alongside the regions it depends on (a pipeline along the
// DAG) instead of waiting for all its inputs first; and the computing
// wavefront issues no global load after the staging, so no batch waits for
// memory except for an input not yet published.  Each row folds its terms
// in ascending column order and divides by its diagonal -- the sequential
// definition's arithmetic, so results are bit-identical to forward
// substitution.  SpMV rows run as the fused executor's items (entry stream,
// x read through the caches first), up to 64 per wavefront.
// No multiply-add contraction in this file.
#pragma clang fp contract(off)

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
template <typename T>
__device__ void region_rows(const TsArgs& a, const RegionArgs& r, int item, int q0, int q1, int b0, int b1,
                            char* lds, unsigned long long* tr) {
  const int R = r.rows_max;
  const RegionLds<T> L = carve<T>(lds, R, r.entries_max, r.ext_max, r.batches_max);
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ B = static_cast<const T*>(a.B);
  T* X = static_cast<T*>(a.X);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nr = q1 - q0;
  const int x0 = r.ext_ptr[item];
  const int nx = r.ext_ptr[item + 1] - x0;
  // stage the region's rows (an entry's code becomes its x slot)
  for (int k = tid; k < nr; k += kRegionThreads) {
    const int id = a.order[q0 + k];
    const int2 rg = reinterpret_cast<const int2*>(a.qrng)[q0 + k];
    const int oo = r.roff[q0 + k];
    const int cnt = rg.y - rg.x;
    RowHead<T> h;
#pragma unroll
    for (int u = 0; u < kRegionAhead; ++u) {
      h.v[u] = T(0);
      h.s[u] = uint16_t(L.zero);
    }
    for (int u = 0; u < cnt; ++u) {
      const int code = r.code[rg.x + u];
      const T v = dev::ld_stream(Lv + rg.x + u);
      const uint16_t slot = uint16_t((code & 0x8000) ? R + (code & 0x7fff) : code);
      if (u < kRegionAhead) {
        h.v[u] = v;
        h.s[u] = slot;
      } else {
        L.ov[oo + u - kRegionAhead] = v;
        L.oc[oo + u - kRegionAhead] = slot;
      }
    }
    h.b = B[id];
    h.d = dev::ld_stream(Lv + rg.y);
    h.id = id;
    h.oo = uint16_t(oo);
    h.on = uint16_t(cnt > kRegionAhead ? cnt - kRegionAhead : 0);
    L.head[k] = h;
  }
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
  if (wid == 1) {
    // the poller: its first W lanes watch inputs lane, lane + W, ... in
    // first-use order (W = r.poll_lanes), backing off r.poll_sleep after a
    // round in which none of them became final
    const int W = r.poll_lanes;
    int k = lane < W ? lane : nx;
    int32_t spins = 0;
    for (;;) {
      if (__ballot(k < nx) == 0) break;
      const T v = k < nx ? ld_co(X + L.xc[k]) : T(0);
      const bool got = k < nx && !is_pending(v);
      if (got) {
        lds_put(L.xa + R + k, v);
        k += W;
      }
      if (!dev::all_poll_round(spins, a.ls)) {
        // watchdog: release every input still pending so the region drains
        for (int q = lane; q < nx; q += 64) lds_put(L.xa + R + q, T(0));
        break;
      }
      if (__ballot(got) == 0)
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
        if (a.rtrace) dev::stamp_publish(a.rtrace, true, c.id);
        st_co(X + c.id, xk);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Claim loop, one block of two wavefronts: regions in topological order,
// SpMV items (up to 256 rows, 64 per wavefront and pass) after them.  With col_units
// > 1, ticket t is column t % col_units of item t / col_units (one chain of
// the items per right-hand side).
template <typename T>
__global__ __launch_bounds__(kRegionThreads) void k_ts_region(TsArgs a, RegionArgs r) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int32_t ticket;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  dev::reset_next_launch(a.ls);
  const int nc = a.col_units > 1 ? a.col_units : 1;
  const int total = a.n_work * nc;
  if (wid == 0) {
    const int t = dev::claim(a.ls, lane);
    if (lane == 0) ticket = t;
  }
  __syncthreads();
  for (;;) {
    const int t = ticket;
    __syncthreads();
    if (t >= total) break;
    // the next ticket's atomic is in flight while this item runs (the
    // item's first loads wait for it too; it is converted at the end)
    int32_t next_raw = 0;
    if (wid == 0) next_raw = dev::claim_issue(a.ls, lane);
    const int u = t / nc, c = t - u * nc;
    const int item = a.item_list ? a.item_list[u] : u;
    TsArgs ac = a;
    if (nc > 1) {
      ac.B = static_cast<const T*>(a.B) + size_t(c) * size_t(a.ldb);
      ac.X = static_cast<T*>(a.X) + size_t(c) * size_t(a.ldx);
      if (a.Y) ac.Y = static_cast<T*>(a.Y) + size_t(c) * size_t(a.ldy);
    }
    const int q0 = a.item_ptr[item], q1 = a.item_ptr[item + 1];
    const int bt0 = r.batch_ptr[item], bt1 = r.batch_ptr[item + 1];
    unsigned long long* tr = a.trace ? a.trace + size_t(item) * kTraceItemWords : nullptr;
    if (tr && tid == 0) {
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      tr[0] = t0;
      tr[1] = t0;
      tr[2] = t0;
      atomicAdd(tr + 4, 1ull);
    }
    if (bt1 > bt0) {
      region_rows<T>(ac, r, item, q0, q1, bt0, bt1, lds, tr);
      __syncthreads();
      if (tr && tid == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
    } else {
      // SpMV rows, 64 per wavefront and pass: rows [0, 64) on wavefront 0,
      // [64, 128) on wavefront 1, [128, 192) on wavefront 0, ...
      for (int s0 = q0 + 64 * wid; s0 < q1; s0 += 128) {
        const int s1 = min(q1, s0 + 64);
        const bool mine = lane < s1 - s0;
        const int id = mine ? a.order[s0 + lane] : 0;
        const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[s0 + lane] : make_int2(0, 0);
        auto* w = reinterpret_cast<dev::WaveLds<T>*>(lds) + wid;
        item_stream_rows<T, false, 3>(ac, s0, s1, lane, *w, nullptr, id, rg);
      }
      __syncthreads();  // both halves' inputs observed and rows stored
      if (tr && tid == 0) {
        const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
        tr[2] = t1;
        tr[3] = t1;
      }
    }
    if (wid == 0) {
      const int tn = dev::claim_ticket(a.ls, next_raw);
      if (lane == 0) ticket = tn;
    }
    __syncthreads();
  }
}

template <typename K>
int occ64(K kernel, size_t lds) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel), kRegionThreads, lds) !=
      hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

size_t region_kernel_lds(const RegionArgs& r, int dtype) {
  const int vb = dtype == 0 ? 8 : 4;
  const size_t reg = region_lds_bytes(r.rows_max, r.entries_max, r.ext_max, r.batches_max, vb);
  const size_t sp = 2 * (dtype == 0 ? sizeof(dev::WaveLds<double>) : sizeof(dev::WaveLds<float>));
  return reg > sp ? reg : sp;
}

int occupancy_region(const RegionArgs& r, int dtype) {
  const size_t lds = region_kernel_lds(r, dtype);
  return dtype == 0 ? occ64(k_ts_region<double>, lds) : occ64(k_ts_region<float>, lds);
}

hipError_t launch_ts_region(const TsArgs& a, const RegionArgs& r, int dtype, int grid, hipStream_t st) {
  if (!a.order || !a.qrng || !a.item_ptr || !r.batch || !r.batch_ptr || !r.ext_ptr || !r.roff || !r.code)
    return hipErrorInvalidValue;
  const size_t lds = region_kernel_lds(r, dtype);
  if (dtype == 0) hipLaunchKernelGGL(k_ts_region<double>, dim3(grid), dim3(kRegionThreads), lds, st, a, r);
  else hipLaunchKernelGGL(k_ts_region<float>, dim3(grid), dim3(kRegionThreads), lds, st, a, r);
  return hipGetLastError();
}

}  // namespace sf
