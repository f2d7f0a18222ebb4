// Work-item building blocks of the SpTRSV -> SpMV executors, shared by the
// fused executor and its baselines (k_ts.hip) and by the fused refinement
// (k_rfused.hip): the entry stream over an item's rows (one right-hand
// side) and the multi-RHS units (KB lanes per row, interleaved blocks).
// Included inside namespace sf's anonymous namespace of each kernel file;
// every file that includes it keeps multiply-add contraction off.
#pragma once

#include "stream.h"

namespace sf {
namespace {

using dev::is_pending;
using dev::kWaves;
using dev::ld_co;
using dev::ld_stream;
using dev::poll_value;
using dev::publishable;
using dev::st_co;
using dev::stream_accumulate;
using dev::WaveLds;

// Trace mode (a.trace != nullptr): per item, timestamps of the 100 MHz
// real-time counter at the start of processing, once the item's indices and
// values are loaded, once every x it reads is ready (after the last wait)
// and at the end, and a count of its runs; per iteration, a stamp taken
// just before its value is published and a count of its publications
// (dev::stamp_publish).  The host checks from them that every item and every
// iteration ran exactly once and that every value was published before the
// wait of each item reading it returned.
__device__ __forceinline__ unsigned long long* trace_slots(const TsArgs& a, int it) {
  return (a.trace && it >= 0) ? a.trace + size_t(it) * kTraceItemWords : nullptr;
}

// Process one item (rows order[q0..q1), q1 - q0 <= 64) of SpTRSV rows
// (TRSV = true) or SpMV rows.  VEC selects how x is read (stream.h): 2 in
// the fused executor (readiness protocol), 1 in the level-set baseline
// (after a grid barrier), 0 in the unfused SpMV (x final before the launch).
// item_stream_rows takes each lane's row id and CSR range (order[q0 + lane]
// and qrng[q0 + lane]) already loaded; item_stream loads them itself.
template <typename T, bool TRSV, int VEC>
__device__ __forceinline__ void item_stream_rows(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w,
                                                 unsigned long long* tr, int id, int2 rg) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const T* __restrict__ val = static_cast<const T*>(TRSV ? a.Lv : a.Av);
  T* X = static_cast<T*>(a.X);
  const int row = TRSV ? id : id - a.n;
  // the row's range comes with its claim position (no row-pointer round trip);
  // an SpTRSV range stops before the diagonal, which sits at r1
  const int r0 = rg.x, r1 = rg.y;
  T acc = T(0), dii = T(1);
  if (TRSV && mine) {
    acc = static_cast<const T*>(a.B)[row];
    dii = ld_stream(val + r1);
  }
  acc = stream_accumulate<T, TRSV, VEC, false>(nr, r0, r1 - r0, acc, TRSV ? a.Lci : a.Aci, nullptr, val, X,
                                               lane, w, a.ls, tr);
  if (a.rtrace) dev::stamp_publish(a.rtrace, mine, id);
  if (mine) {
    if constexpr (TRSV) st_co(X + row, publishable(acc / dii));
    else __builtin_nontemporal_store(acc, static_cast<T*>(a.Y) + row);
  }
  if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
}

// Prefix fusion (level items; a.apre set): an SpTRSV item whose rows also
// fold their SpMV row's prefix and publish it to Y (read back by the SpMV
// row, which continues the fold: A's entry order is kept, so y is the
// sequential definition's bit for bit).  a0: the lane's row's first prefix
// position in A, or -1; the diagonal A_ii closes the prefix at a0 + (row's
// off-diagonal count), multiplied by the published x_i.
template <typename T, int VEC>
__device__ __forceinline__ void item_stream_rows_pre(const TsArgs& a, int q0, int q1, int lane,
                                                     dev::WaveLdsPre<T>& w, unsigned long long* tr, int id,
                                                     int2 rg, int a0) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const T* __restrict__ val = static_cast<const T*>(a.Lv);
  const T* __restrict__ aval = static_cast<const T*>(a.Av);
  T* X = static_cast<T*>(a.X);
  const int r0 = rg.x, r1 = rg.y;
  T acc = T(0), dii = T(1), acc2 = T(0);
  if (mine) {
    acc = static_cast<const T*>(a.B)[id];
    dii = ld_stream(val + r1);
  }
  acc = dev::stream_accumulate_pre<T, VEC>(nr, r0, r1 - r0, mine ? a0 : -1, acc, acc2, a.Lci, val, aval, X, lane,
                                           w, a.ls, tr);
  if (a.rtrace) dev::stamp_publish(a.rtrace, mine, id);
  if (mine) {
    const T x = publishable(acc / dii);
    st_co(X + id, x);
    if (a0 >= 0) st_co(static_cast<T*>(a.Y) + id, publishable(acc2 + ld_stream(aval + a0 + (r1 - r0)) * x));
  }
  if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
}

// SpMV rows under prefix fusion: a row with a folded prefix (qrng.x < 0,
// encoding -(first position past the prefix + 1)) starts from its partial
// sum in Y; the others from 0, as item_stream_rows.
template <typename T, int VEC>
__device__ __forceinline__ void item_spmv_rows_from(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w,
                                                    unsigned long long* tr, int id, int2 rg) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const int row = id - a.n;
  T* Y = static_cast<T*>(a.Y);
  const bool pre = mine && rg.x < 0;
  const int r0 = pre ? -rg.x - 1 : rg.x;
  T acc = dev::stream_accumulate_from<T, VEC>(nr, r0, rg.y - r0, pre ? Y + row : nullptr, a.Aci,
                                              static_cast<const T*>(a.Av), static_cast<const T*>(a.X), lane, w,
                                              a.ls, tr);
  if (a.rtrace) dev::stamp_publish(a.rtrace, mine, id);
  if (mine) __builtin_nontemporal_store(acc, Y + row);
  if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
}

template <typename T, bool TRSV, int VEC>
__device__ __forceinline__ void item_stream(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w,
                                            int it = -1) {
  const bool mine = lane < q1 - q0;
  unsigned long long* tr = trace_slots(a, it);
  if (tr && lane == 0) tr[0] = __builtin_amdgcn_s_memrealtime();
  const int id = mine ? a.order[q0 + lane] : 0;
  const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[q0 + lane] : make_int2(0, 0);
  item_stream_rows<T, TRSV, VEC>(a, q0, q1, lane, w, tr, id, rg);
}

// Coarsened SpTRSV item (rows on several local wavefronts, sorted by local
// wavefront): dev::chunk_solve (stream.h) over the rows' off-diagonals.
// Each lane's row, CSR range and local wavefront come loaded, with the
// item's last local wavefront.
template <typename T>
__device__ __forceinline__ void item_chunk_rows(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w, T* xl,
                                                unsigned long long* tr, int row, int2 rg, int myloc, int maxloc) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const T* __restrict__ val = static_cast<const T*>(a.Lv);
  const int r0 = rg.x, r1 = rg.y;  // off-diagonals; the diagonal sits at r1
  const T acc = mine ? static_cast<const T*>(a.B)[row] : T(0);
  const T dii = mine ? ld_stream(val + r1) : T(1);
  dev::chunk_solve<T, false>(nr, r0, r1 - r0, myloc, maxloc, acc, dii, a.Lci, nullptr, val, a.eloc,
                             static_cast<T*>(a.X), row, lane, w, xl, a.ls, tr, a.rtrace);
  if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
}

// Work item `it` of a kernel whose items run in claim order (item_list
// maps the claim index u to the item when given): its claim positions
// [q0, q1).  Every lane loads them (uniform addresses).
__device__ __forceinline__ void item_range(const TsArgs& a, int u, int& it, int& q0, int& q1) {
  it = a.item_list ? a.item_list[u] : u;
  q0 = a.item_ptr[it];
  q1 = a.item_ptr[it + 1];
}

// ------------------------------------------------------------- k > 1 ------
// KB lanes per row, one lane per right-hand side of the block, 64 / KB rows
// per wavefront.  B, the solution xi (filled with the pending pattern before
// the launch) and Y are in the interleaved block layout: row j of block b
// holds its KB values contiguously at [(b * rows + j) * KB], so a lane's
// gather of x_j and its reads and writes of row i are coalesced across the
// row's lanes.  Each lane folds its row's terms in ascending entry order
// (b_i minus, or 0 plus, each rounded product).

// One row of the unfused SpMV over finished x, kU entries at a time (their
// indices and values, then their x, loaded together through the caches).
constexpr int kU = 8;
template <typename T, int KB>
__device__ __forceinline__ T row_final(const int32_t* __restrict__ col, const T* __restrict__ val, const T* xi,
                                       int p0, int p1, int c) {
  T acc = T(0);
  for (int c0 = p0; c0 < p1; c0 += kU) {
    int j[kU];
    T v[kU], xv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool h = c0 + u < p1;
      j[u] = h ? col[c0 + u] : -1;
      v[u] = h ? val[c0 + u] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) xv[u] = j[u] >= 0 ? xi[size_t(j[u]) * KB + c] : T(0);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (j[u] < 0) break;
      acc = acc + v[u] * xv[u];
    }
  }
  return acc;
}

// A unit of the multi-RHS plan: up to 64 / KB rows of one kind, claim
// positions [q0, q1).  Row meta (its index and CSR range, both with the
// claim position) takes one round trip.  Units whose rows have at most
// kShort entries load them directly in each lane; otherwise, a chunk of
// S::CH entries per row at a time, the row's KB lanes stage its column
// indices and values in LDS with one round of loads (lane c takes entries
// c, c + KB, ...).  Every lane then gathers its column of x for up to kUx
// entries at once and waits for the pending ones of the whole wavefront
// together (dev::wait_ready on offsets into the block's interleaved x).  Products are folded in
// ascending entry order.  POLL = false (level set): x was written before a
// grid barrier and is read device-coherently without waiting.
template <int KB>
struct MultiShape {
  static constexpr int NE = KB <= 8 ? 8 : 4;  // entries each lane stages per chunk
  static constexpr int CH = KB * NE;          // entries of one row per chunk
};
template <typename T, int KB>
struct MultiLds {
  int32_t col[64 * MultiShape<KB>::NE];
  T val[64 * MultiShape<KB>::NE];
};
constexpr int kUx = 8;     // x gathers per lane in flight per wait round
constexpr int kShort = 8;  // rows up to this long skip the LDS staging

template <typename T, int KB, bool POLL>
__device__ __forceinline__ void unit_multi(const TsArgs& a, int q0, int q1, int blk, int lane,
                                           MultiLds<T, KB>& w, int next = -1, int2* next_rg = nullptr) {
  using S = MultiShape<KB>;
  const int g = lane / KB, c = lane % KB;
  const int q = q0 + g;
  const bool act = q < q1;
  const int id = act ? a.order[q] : 0;
  // an SpTRSV range stops before the diagonal
  const int2 rg = act ? reinterpret_cast<const int2*>(a.qrng)[q] : make_int2(0, 0);
  // the next unit's range, loaded once its ticket has arrived (it returns
  // before the row meta above) and used after this unit
  if (next_rg) *next_rg = next >= 0 ? a.unit_rng[next] : make_int2(0, 0);
  const bool trsv = __shfl(id, 0, 64) < a.n;  // a unit holds rows of one kind
  const T* __restrict__ val = static_cast<const T*>(trsv ? a.Lv : a.Av);
  const int32_t* __restrict__ col = trsv ? a.Lci : a.Aci;
  const size_t xoff = size_t(blk) * size_t(a.n) * KB;
  T* xb = static_cast<T*>(a.xi) + xoff;
  T acc = T(0), dii = T(1);
  if (trsv && act) {
    acc = static_cast<const T*>(a.B)[xoff + size_t(id) * KB + c];
    dii = ld_stream(val + rg.y);
  }
  const int len = rg.y - rg.x;
  int maxlen = len;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, d, 64));
  if (maxlen <= kShort) {
    // short rows: each lane loads its row's indices and values itself (the
    // row's lanes read the same addresses), then gathers its column of x
    int idx[kShort];
    T v[kShort], xv[kShort];
#pragma unroll
    for (int u = 0; u < kShort; ++u) {
      const bool h = u < len;
      idx[u] = h ? ld_stream(col + rg.x + u) : -1;
      v[u] = h ? ld_stream(val + rg.x + u) : T(0);
    }
#pragma unroll
    for (int u = 0; u < kShort; ++u) {
      idx[u] = idx[u] >= 0 ? idx[u] * KB + c : -1;
      xv[u] = idx[u] >= 0 ? ld_co(xb + idx[u]) : T(0);
    }
    if constexpr (POLL) dev::wait_ready<T, kShort, 64>(xb, idx, xv, lane, a.ls);
#pragma unroll
    for (int u = 0; u < kShort; ++u) {
      if (idx[u] < 0) break;
      const T pr = v[u] * xv[u];
      acc = trsv ? acc - pr : acc + pr;
    }
  }
  const int slice = g * S::CH;
  for (int base = 0; maxlen > kShort && base < maxlen; base += S::CH) {
#pragma unroll
    for (int e = 0; e < S::NE; ++e) {
      const int u = base + c + KB * e;
      if (u < len) {
        w.col[slice + c + KB * e] = ld_stream(col + rg.x + u);
        w.val[slice + c + KB * e] = ld_stream(val + rg.x + u);
      }
    }
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(S::CH, len - base);  // this row's entries in the chunk (may be <= 0)
    int wcnt = cnt;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wcnt = max(wcnt, __shfl_xor(wcnt, d, 64));
    for (int r0 = 0; r0 < wcnt; r0 += kUx) {
      int idx[kUx];
      T xv[kUx];
#pragma unroll
      for (int u = 0; u < kUx; ++u) {
        idx[u] = r0 + u < cnt ? w.col[slice + r0 + u] * KB + c : -1;
        xv[u] = idx[u] >= 0 ? ld_co(xb + idx[u]) : T(0);
      }
      if constexpr (POLL) dev::wait_ready<T, kUx, 64>(xb, idx, xv, lane, a.ls);
#pragma unroll
      for (int u = 0; u < kUx; ++u) {
        if (idx[u] < 0) break;
        const T pr = w.val[slice + r0 + u] * xv[u];
        acc = trsv ? acc - pr : acc + pr;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (act) {
    if (trsv) st_co(xb + size_t(id) * KB + c, publishable(acc / dii));
    else __builtin_nontemporal_store(acc, static_cast<T*>(a.Y) + size_t(blk) * size_t(a.m) * KB +
                                              size_t(id - a.n) * KB + c);
  }
}

}  // namespace
}  // namespace sf
