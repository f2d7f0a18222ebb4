// Mixed-precision refinement of x = L^{-1} b, with y = A x, as one fused
// schedule (gfx950).
//
// Staged, the refinement is a chain of kernels: an FP32 substitution
// (L32 x0 = fl32(b)), then per correction t an FP64 residual
// r = b - L64 x and an FP32 substitution L32 d_t = fl32(r), x += d_t, and at
// the end y = A64 x and the residual norm.  Row i of every stage needs only
// rows j <= i of the previous stages (r_i reads x_j for the stored j of row
// i, the diagonal included), i.e. the dependence matrix between consecutive
// stages is the pattern of L and every stage's DAG is L's: the whole chain
// composes into one DAG walk over L's schedule, the paper's fusion of
// loop-carried-dependence kernels with F = I (interleaved packing).  A row
// gathers, for each stored j, one tuple (x0_j, d_1j, ..., d_NC,j) -- all
// stage values of row j -- and computes all its stages in registers:
//     s_t  = sum_j fl32(L32_ij v_t,j)      (FP32, ascending j, from 0)
//     rh_t = sum_j L64_ij X_{t-1},j        (FP64, ascending j, from 0)
//     x0_i  = fl32(fl32(fl32(b_i) - s_0) / L32_ii),  X_0 = 0 + x0
//     r     = b_i - (rh_t + L64_ii X_{t-1},i),   d_t,i = fl32(fl32(fl32(r) - s_t) / L32_ii)
//     X_t   = X_{t-1} + d_t,i                  (FP64)
// where X_t,j is rebuilt from the tuple in the same order, and finally the
// residual b_i - (rh_{NC+1} + L64_ii X_NC,i) for the norm.  The row then
// publishes its tuple (one coherent vector store; every component carries
// the FP32 pending pattern until then) and x_i = X_NC,i (FP64, the flag the
// SpMV rows wait on).  SpMV rows are the fused executor's, over x.  Each
// FP32 substitution sums its off-diagonal products first and subtracts the
// sum from the rounded right-hand side, so no stage sum needs a value of the
// row's own chain; this order is the refinement's definition (the oracle's
// orc_refine), and results are bit-identical to it.
//
// One right-hand side: level items through an entry stream (all entries of
// an item dealt to the lanes, products into LDS, the owner lane folds).
// Several: the multi-RHS units (KB lanes per row, one per right-hand side,
// interleaved blocks; each lane folds its own column).
// No multiply-add contraction in this file.
#pragma clang fp contract(off)

#include "ts_items.h"

namespace sf {
namespace {

using dev::is_pending;
using dev::kPass;
using dev::kRounds;
using dev::kWaves;
using dev::ld_stream;
using dev::publishable;
using dev::st_co;

// A row's stage values: x0, d_1 .. d_NC (S4 = 2 or 4 floats, padded),
// stored as H = S4 / 2 64-bit halves.  Layout of a block of KB right-hand
// sides: half h of row j, column c at 64-bit word (j * H + h) * KB + c, so
// the KB lanes of a row read each half as one contiguous run.  Each half is
// read and written with one device-coherent 64-bit access; its floats carry
// the pending pattern until published.
template <int NC>
struct Tup {
  static constexpr int S4 = NC <= 1 ? 2 : 4;
  static constexpr int H = S4 / 2;
  float v[S4];
};

template <int NC, int KB>
__device__ __forceinline__ Tup<NC> tup_load(const unsigned long long* tb, int64_t j, int c) {
  Tup<NC> t;
#pragma unroll
  for (int h = 0; h < Tup<NC>::H; ++h) {
    const unsigned long long u = dev::ld_co(tb + (j * Tup<NC>::H + h) * KB + c);
    t.v[2 * h] = __builtin_bit_cast(float, static_cast<unsigned int>(u));
    t.v[2 * h + 1] = __builtin_bit_cast(float, static_cast<unsigned int>(u >> 32));
  }
  return t;
}

template <int NC, int KB>
__device__ __forceinline__ void tup_store(unsigned long long* tb, int64_t j, int c, const Tup<NC>& t) {
#pragma unroll
  for (int h = 0; h < Tup<NC>::H; ++h) {
    const unsigned long long u = static_cast<unsigned long long>(__builtin_bit_cast(unsigned int, t.v[2 * h])) |
                                 (static_cast<unsigned long long>(__builtin_bit_cast(unsigned int, t.v[2 * h + 1]))
                                  << 32);
    st_co(tb + (j * Tup<NC>::H + h) * KB + c, u);
  }
}

template <int NC>
__device__ __forceinline__ bool tup_pending(const Tup<NC>& t) {
  bool p = false;
#pragma unroll
  for (int k = 0; k <= NC; ++k) p = p || is_pending(t.v[k]);
  return p;
}

// Wait until every tuple tp[e] of a column j[e] >= 0 is published (every
// lane re-reads its pending tuples each round; the watchdog bounds the wait).
template <int NC, int KB, int R>
__device__ __forceinline__ void tup_wait(const unsigned long long* tb, const int (&j)[R], int c, Tup<NC> (&tp)[R],
                                         const LaunchState& ls) {
  int32_t spins = 0;
  for (;;) {
    bool any = false;
#pragma unroll
    for (int e = 0; e < R; ++e) any = any || (j[e] >= 0 && tup_pending<NC>(tp[e]));
    if (__ballot(any) == 0) return;
#pragma unroll
    for (int e = 0; e < R; ++e)
      if (j[e] >= 0 && tup_pending<NC>(tp[e])) tp[e] = tup_load<NC, KB>(tb, j[e], c);
    if (!dev::all_poll_round(spins, ls)) return;
  }
}

// The row's chain from its stage sums; returns the tuple, the final x and
// the final residual.
template <int NC>
__device__ __forceinline__ Tup<NC> rf_chain(double bi, float l32d, double l64d, const float (&sg)[NC + 1],
                                            const double (&rh)[NC + 1], double& X, double& rfin) {
  Tup<NC> t;
#pragma unroll
  for (int k = 0; k < Tup<NC>::S4; ++k) t.v[k] = 0.0f;
  const float c0 = float(bi);
  const float x0 = publishable((c0 - sg[0]) / l32d);
  t.v[0] = x0;
  X = 0.0 + double(x0);
#pragma unroll
  for (int k = 1; k <= NC; ++k) {
    const double r = bi - (rh[k - 1] + l64d * X);
    const float ck = float(r);
    const float d = publishable((ck - sg[k]) / l32d);
    t.v[k] = d;
    X = X + double(d);
  }
  rfin = bi - (rh[NC] + l64d * X);
  return t;
}

// The terms of one stored entry (value pair v32 / v64, column tuple tp):
// FP32 products of every stage and FP64 products of every residual.
template <int NC>
__device__ __forceinline__ void rf_terms(float v32, double v64, const Tup<NC>& tp, float (&pf)[NC + 1],
                                         double (&pd)[NC + 1]) {
  double X = 0.0 + double(tp.v[0]);
  pf[0] = v32 * tp.v[0];
#pragma unroll
  for (int k = 1; k <= NC; ++k) {
    pd[k - 1] = v64 * X;
    pf[k] = v32 * tp.v[k];
    X = X + double(tp.v[k]);
  }
  pd[NC] = v64 * X;
}

// ---------------------------------------------------- one right-hand side --
template <int NC>
struct RfLds {
  int32_t pos[kPass];
  float pf[NC + 1][kPass];
  double pd[NC + 1][kPass];
};

// The SpTRSV rows order[q0..q1) of a level item (independent rows): every
// stored off-diagonal of the item is dealt to the lanes, kRounds per lane,
// with its index, both values and its column's tuple loaded in one round;
// the terms go to LDS and each row's lane folds its own in ascending order.
template <int NC>
__device__ __forceinline__ void rf_rows(const RfArgs& a, int q0, int q1, int lane, RfLds<NC>& w, int id, int2 rg,
                                       unsigned long long* smax) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  int len = mine ? rg.y - rg.x : 0;  // off-diagonals; the diagonal sits at rg.y
  int incl = len;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int off = incl - len;
  const int total = __shfl(incl, 63, 64);
  unsigned long long* tb = a.tup;
  float sg[NC + 1];
  double rh[NC + 1];
#pragma unroll
  for (int k = 0; k <= NC; ++k) {
    sg[k] = 0.0f;
    rh[k] = 0.0;
  }
  for (int base = 0; base < total; base += kPass) {
    if (mine) {
      const int lo = max(off, base), hi = min(off + len, base + kPass);
      for (int t = lo; t < hi; ++t) w.pos[t - base] = rg.x + (t - off);
    }
    __builtin_amdgcn_wave_barrier();
    int j[kRounds];
    float v32[kRounds];
    double v64[kRounds];
    Tup<NC> tp[kRounds];
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      j[e] = -1;
      v32[e] = 0.0f;
      v64[e] = 0.0;
      if (k < total) {
        const int p = w.pos[k - base];
        j[e] = ld_stream(a.ts.Lci + p);
        v32[e] = ld_stream(a.L32 + p);
        v64[e] = ld_stream(static_cast<const double*>(a.ts.Lv) + p);
      }
    }
#pragma unroll
    for (int e = 0; e < kRounds; ++e)
      if (j[e] >= 0) tp[e] = tup_load<NC, 1>(tb, j[e], 0);
    tup_wait<NC, 1, kRounds>(tb, j, 0, tp, a.ts.ls);
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      if (k < total) {
        float pf[NC + 1];
        double pd[NC + 1];
        rf_terms<NC>(v32[e], v64[e], tp[e], pf, pd);
#pragma unroll
        for (int s = 0; s <= NC; ++s) {
          w.pf[s][k - base] = pf[s];
          w.pd[s][k - base] = pd[s];
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (mine) {
      const int lo = max(off, base) - base;
      const int hi = min(off + len, base + kPass) - base;
      // ascending order, one rounding per term; the LDS reads of four
      // entries are issued before their additions
      int t = lo;
      for (; t + 4 <= hi; t += 4) {
        float f[4][NC + 1];
        double d[4][NC + 1];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int s = 0; s <= NC; ++s) {
            f[u][s] = w.pf[s][t + u];
            d[u][s] = w.pd[s][t + u];
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int s = 0; s <= NC; ++s) {
            sg[s] = sg[s] + f[u][s];
            rh[s] = rh[s] + d[u][s];
          }
      }
      for (; t < hi; ++t) {
#pragma unroll
        for (int s = 0; s <= NC; ++s) {
          sg[s] = sg[s] + w.pf[s][t];
          rh[s] = rh[s] + w.pd[s][t];
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  double bi = 0.0, l64d = 1.0;
  float l32d = 1.0f;
  if (mine) {
    bi = a.B[id];
    l32d = ld_stream(a.L32 + rg.y);
    l64d = ld_stream(static_cast<const double*>(a.ts.Lv) + rg.y);
  }
  double X = 0.0, rfin = 0.0;
  const Tup<NC> t = rf_chain<NC>(bi, l32d, l64d, sg, rh, X, rfin);
  if (mine) {
    tup_store<NC, 1>(tb, id, 0, t);
    st_co(static_cast<double*>(a.ts.X) + id, publishable(X));
  }
  // per-wave maxima, then one atomic from lane 0
  double mr = mine ? fabs(rfin) : 0.0, mb = mine ? fabs(bi) : 0.0;
  unsigned long long ur = (unsigned long long)__double_as_longlong(mr);
  unsigned long long ub = (unsigned long long)__double_as_longlong(mb);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    ur = max(ur, (unsigned long long)__shfl_xor((long long)ur, d, 64));
    ub = max(ub, (unsigned long long)__shfl_xor((long long)ub, d, 64));
  }
  if (lane == 0) {  // the block's maxima in LDS; one device atomic per block at the end
    if (ur) atomicMax(smax, ur);
    if (ub) atomicMax(smax + 1, ub);
  }
}

// A block's |r| and |b| maxima (2 per column, in LDS) into the device
// accumulators: one atomic per word and block instead of one per row group.
__device__ __forceinline__ void flush_maxima(unsigned long long* mx, const unsigned long long* smax, int words) {
  __syncthreads();
  for (int k = threadIdx.x; k < words; k += blockDim.x)
    if (smax[k]) __hip_atomic_fetch_max(mx + k, smax[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NC>
union RfWaveLds {
  RfLds<NC> rf;
  dev::WaveLds<double> sp;
};

// Claim loop: level items in joint order (SpTRSV items with their stages,
// SpMV items over the published x), the next ticket claimed ahead.
template <int NC>
__global__ __launch_bounds__(kBlockThreads) void k_rf_stream(RfArgs a) {
  __shared__ RfWaveLds<NC> lds[kWaves];
  __shared__ unsigned long long smax[2];
  const int lane = threadIdx.x & 63;
  RfWaveLds<NC>& w = lds[threadIdx.x >> 6];
  const TsArgs& ts = a.ts;
  if (threadIdx.x < 2) smax[threadIdx.x] = 0ull;
  __syncthreads();
  dev::reset_next_launch(ts.ls);
  int t = dev::claim(ts.ls, lane);
  while (t < ts.n_work) {
    const int tn = dev::claim(ts.ls, lane);
    const int it = ts.item_list ? ts.item_list[t] : t;
    const int q0 = ts.item_ptr[it], q1 = ts.item_ptr[it + 1];
    const bool mine = lane < q1 - q0;
    const int id = mine ? ts.order[q0 + lane] : 0;
    const int2 rg = mine ? reinterpret_cast<const int2*>(ts.qrng)[q0 + lane] : make_int2(0, 0);
    if (__shfl(id, 0, 64) < ts.n) rf_rows<NC>(a, q0, q1, lane, w.rf, id, rg, smax);
    else item_stream_rows<double, false, 2>(ts, q0, q1, lane, w.sp, nullptr, id, rg);
    t = tn;
  }
  flush_maxima(a.maxabs, smax, 2);
}

// ------------------------------------------------ several right-hand sides --
// A unit of SpTRSV rows (64 / KB rows, KB lanes each, lane c = column c of
// block blk): the lane walks its row's entries kUx at a time (indices and
// both values, then the column tuples of its right-hand side, waited for
// together) and folds the terms of every stage in ascending order.
// Entries a row's KB lanes stage per chunk (lane c takes entries c, c + KB,
// ...): the indices and both values of S::CH entries in one round of loads.
template <int KB>
struct RfShape {
  static constexpr int NE = KB <= 8 ? 8 : 4;
  static constexpr int CH = KB * NE;
};
template <int KB>
struct RfMultiLds {
  int32_t col[64 * RfShape<KB>::NE];
  float v32[64 * RfShape<KB>::NE];
  double v64[64 * RfShape<KB>::NE];
};

template <int NC, int KB>
__device__ __forceinline__ void rf_fold_entries(const RfArgs& a, const unsigned long long* tb, int c, int cnt,
                                                const int32_t* col, const float* v32, const double* v64,
                                                float (&sg)[NC + 1], double (&rh)[NC + 1], int wmax) {
  for (int r0 = 0; r0 < wmax; r0 += kUx) {
    int j[kUx];
    Tup<NC> tp[kUx];
#pragma unroll
    for (int u = 0; u < kUx; ++u) {
      j[u] = r0 + u < cnt ? col[r0 + u] : -1;
      if (j[u] >= 0) tp[u] = tup_load<NC, KB>(tb, j[u], c);
    }
    tup_wait<NC, KB, kUx>(tb, j, c, tp, a.ts.ls);
#pragma unroll
    for (int u = 0; u < kUx; ++u) {
      if (j[u] < 0) break;
      float pf[NC + 1];
      double pd[NC + 1];
      rf_terms<NC>(v32[r0 + u], v64[r0 + u], tp[u], pf, pd);
#pragma unroll
      for (int s = 0; s <= NC; ++s) {
        sg[s] = sg[s] + pf[s];
        rh[s] = rh[s] + pd[s];
      }
    }
  }
}

// A unit of SpTRSV rows (64 / KB rows, KB lanes each, lane c = column c of
// block blk): the row's entries are staged in LDS a chunk at a time (one
// round of loads), then every lane gathers its column's tuples kUx at a
// time, waits for the pending ones and folds the terms of every stage in
// ascending order.
template <int NC, int KB>
__device__ __forceinline__ void rf_unit(const RfArgs& a, int q0, int q1, int blk, int lane, RfMultiLds<KB>& w,
                                       unsigned long long* smax) {
  using S = RfShape<KB>;
  const TsArgs& ts = a.ts;
  const int g = lane / KB, c = lane % KB;
  const int q = q0 + g;
  const bool act = q < q1;
  const int id = act ? ts.order[q] : 0;
  const int2 rg = act ? reinterpret_cast<const int2*>(ts.qrng)[q] : make_int2(0, 0);
  const size_t row0 = size_t(blk) * size_t(ts.n);  // first row of this block in the interleaved arrays
  unsigned long long* tb = a.tup + row0 * KB * Tup<NC>::H;  // this block's tuples
  const double* __restrict__ L64 = static_cast<const double*>(ts.Lv);
  const int len = rg.y - rg.x;
  int maxlen = len;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, d, 64));
  float sg[NC + 1];
  double rh[NC + 1];
#pragma unroll
  for (int k = 0; k <= NC; ++k) {
    sg[k] = 0.0f;
    rh[k] = 0.0;
  }
  const int slice = g * S::CH;
  for (int base = 0; base < maxlen; base += S::CH) {
#pragma unroll
    for (int e = 0; e < S::NE; ++e) {
      const int u = base + c + KB * e;
      if (u < len) {
        w.col[slice + c + KB * e] = ld_stream(ts.Lci + rg.x + u);
        w.v32[slice + c + KB * e] = ld_stream(a.L32 + rg.x + u);
        w.v64[slice + c + KB * e] = ld_stream(L64 + rg.x + u);
      }
    }
    __builtin_amdgcn_wave_barrier();
    const int cnt = min(S::CH, len - base);
    int wcnt = cnt;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wcnt = max(wcnt, __shfl_xor(wcnt, d, 64));
    rf_fold_entries<NC, KB>(a, tb, c, cnt, w.col + slice, w.v32 + slice, w.v64 + slice, sg, rh, wcnt);
    __builtin_amdgcn_wave_barrier();
  }
  const size_t at = (row0 + size_t(id)) * KB + c;
  double bi = 0.0, l64d = 1.0;
  float l32d = 1.0f;
  if (act) {
    bi = a.B[at];  // zero in the padding columns of the last block
    l32d = ld_stream(a.L32 + rg.y);
    l64d = ld_stream(L64 + rg.y);
  }
  double X = 0.0, rfin = 0.0;
  const Tup<NC> t = rf_chain<NC>(bi, l32d, l64d, sg, rh, X, rfin);
  if (act) {
    tup_store<NC, KB>(tb, id, c, t);
    st_co(static_cast<double*>(ts.xi) + at, publishable(X));
  }
  // maxima per column: reduce over the unit's rows of each column (lanes
  // c, c + KB, ...) into the block's LDS maxima
  const int col = blk * KB + c;
  unsigned long long ur = act ? (unsigned long long)__double_as_longlong(fabs(rfin)) : 0ull;
  unsigned long long ub = act ? (unsigned long long)__double_as_longlong(fabs(bi)) : 0ull;
#pragma unroll
  for (int d = 32; d >= KB; d >>= 1) {
    ur = max(ur, (unsigned long long)__shfl_xor((long long)ur, d, 64));
    ub = max(ub, (unsigned long long)__shfl_xor((long long)ub, d, 64));
  }
  if (g == 0 && col < a.nrhs) {
    if (ur) atomicMax(smax + 2 * col, ur);
    if (ub) atomicMax(smax + 2 * col + 1, ub);
  }
}

// Work index t = unit * nblk + block, units in joint order (SpTRSV units
// with their stages, SpMV units over the published interleaved x).
template <int KB>
union RfMultiWaveLds {
  RfMultiLds<KB> rf;
  MultiLds<double, KB> ml;
};

template <int NC, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_rf_multi(RfArgs a) {
  __shared__ RfMultiWaveLds<KB> lds[kWaves];
  __shared__ unsigned long long smax[2 * 64];
  const int lane = threadIdx.x & 63;
  RfMultiWaveLds<KB>& w = lds[threadIdx.x >> 6];
  const TsArgs& ts = a.ts;
  for (int k = threadIdx.x; k < 2 * 64; k += blockDim.x) smax[k] = 0ull;
  __syncthreads();
  dev::reset_next_launch(ts.ls);
  const int total = ts.n_work * ts.nblk;
  int t = dev::claim(ts.ls, lane);
  while (t < total) {
    const int tn = dev::claim(ts.ls, lane);
    const int2 rg = ts.unit_rng[t / ts.nblk];
    const int blk = t % ts.nblk;
    const int id0 = ts.order[rg.x];
    if (id0 < ts.n) rf_unit<NC, KB>(a, rg.x, rg.y, blk, lane, w.rf, smax);
    else unit_multi<double, KB, true>(ts, rg.x, rg.y, blk, lane, w.ml);
    t = tn;
  }
  flush_maxima(a.maxabs, smax, 2 * a.nrhs);
}

template <typename K>
int occ(K kernel) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel), kBlockThreads, 0) !=
      hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

template <int NC>
hipError_t rf_multi_dispatch(const RfArgs& a, int kb, int grid, hipStream_t st) {
#define SF_RM(KB)                                                                          \
  if (kb == KB) {                                                                          \
    hipLaunchKernelGGL((k_rf_multi<NC, KB>), dim3(grid), dim3(kBlockThreads), 0, st, a);  \
    return hipGetLastError();                                                              \
  }
  SF_RM(2) SF_RM(4) SF_RM(8) SF_RM(16) SF_RM(32) SF_RM(64)
#undef SF_RM
  return hipErrorInvalidValue;
}

template <int NC>
int rf_occ(int kb) {
  switch (kb) {
    case 1: return occ(k_rf_stream<NC>);
    case 2: return occ(k_rf_multi<NC, 2>);
    case 4: return occ(k_rf_multi<NC, 4>);
    case 8: return occ(k_rf_multi<NC, 8>);
    case 16: return occ(k_rf_multi<NC, 16>);
    case 32: return occ(k_rf_multi<NC, 32>);
    default: return occ(k_rf_multi<NC, 64>);
  }
}

}  // namespace

int rf_tuple_floats(int nc) { return nc <= 1 ? 2 : 4; }

int occupancy_rfused(int nc, int kb) {
  switch (nc) {
    case 0: return rf_occ<0>(kb);
    case 1: return rf_occ<1>(kb);
    case 2: return rf_occ<2>(kb);
    default: return rf_occ<3>(kb);
  }
}

hipError_t launch_rfused(const RfArgs& a, int nc, int kb, int grid, hipStream_t st) {
  if (!a.ts.order || !a.ts.qrng || !a.tup || !a.B || !a.L32 || !a.ts.Lv || !a.maxabs || nc < 0 || nc > 3)
    return hipErrorInvalidValue;
  if (kb == 1) {
    if (!a.ts.item_ptr || !a.ts.X) return hipErrorInvalidValue;
#define SF_RS(NC) \
  if (nc == NC) hipLaunchKernelGGL(k_rf_stream<NC>, dim3(grid), dim3(kBlockThreads), 0, st, a);
    SF_RS(0) SF_RS(1) SF_RS(2) SF_RS(3)
#undef SF_RS
    return hipGetLastError();
  }
  if (!a.ts.unit_rng || !a.ts.xi || a.ts.nblk < 1) return hipErrorInvalidValue;
  switch (nc) {
    case 0: return rf_multi_dispatch<0>(a, kb, grid, st);
    case 1: return rf_multi_dispatch<1>(a, kb, grid, st);
    case 2: return rf_multi_dispatch<2>(a, kb, grid, st);
    default: return rf_multi_dispatch<3>(a, kb, grid, st);
  }
}

}  // namespace sf
