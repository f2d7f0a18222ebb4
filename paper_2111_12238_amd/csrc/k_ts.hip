// Fused SpTRSV -> SpMV executor and its unfused baseline (gfx950).
//
// One persistent launch runs the whole joint schedule (the two kernels as
// one schedule over their joint DAG).  Each 64-lane wavefront claims work
// items in the joint wavefront order; an item holds up to 64 rows of one
// wavefront and one kind, so its rows are independent.  A SpTRSV row computes
//     x_i = (b_i - sum_{j<i} L_ij x_j) / L_ii
// from the x_j it reads, each observed ready through the value-as-flag
// protocol (dev_common.h), and publishes x_i with one device-coherent store;
// a SpMV row reads every x_j it needs (F = pattern of A) the same way and
// stores y_r = sum_j A_rj x_j.  The diagonal is the last stored entry of each
// row of L (checked by the inspector).
//
// Item processing ("entry stream").  The off-diagonal entries of the item's
// rows are concatenated and dealt to the 64 lanes, kRounds per lane, so a
// single round of independent loads fetches every index, value and x of the
// item (one memory round trip on the critical path whatever the row lengths).
// Each product L_ij * x_j is rounded once into LDS; then the lane that owns
// row i subtracts them from b_i in ascending column order and divides by
// L_ii -- exactly the sequential definition's operations in its order, so
// FP64 results are bit-identical to forward substitution done row by row.
// SpMV rows add their products to 0 the same way.  No multiply-add
// contraction is allowed in this file.
#pragma clang fp contract(off)

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
// values are loaded, once every x it reads is ready, and at the end.
__device__ __forceinline__ unsigned long long* trace_slots(const TsArgs& a, int it) {
  return (a.trace && it >= 0) ? a.trace + size_t(it) * 4 : nullptr;
}

// Process one item (rows order[q0..q1), q1 - q0 <= 64) of SpTRSV rows
// (TRSV = true) or SpMV rows.  VEC selects how x is read (stream.h): 2 in
// the fused executor (readiness protocol), 1 in the level-set baseline
// (after a grid barrier), 0 in the unfused SpMV (x final before the launch).
template <typename T, bool TRSV, int VEC>
__device__ __forceinline__ void item_stream(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w,
                                            int it = -1) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const T* __restrict__ val = static_cast<const T*>(TRSV ? a.Lv : a.Av);
  T* X = static_cast<T*>(a.X);
  unsigned long long* tr = trace_slots(a, it);
  if (tr && lane == 0) tr[0] = __builtin_amdgcn_s_memrealtime();
  const int id = mine ? a.order[q0 + lane] : 0;
  const int row = TRSV ? id : id - a.n;
  // the row's range comes with its claim position (no row-pointer round trip);
  // an SpTRSV range stops before the diagonal, which sits at r1
  const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[q0 + lane] : make_int2(0, 0);
  const int r0 = rg.x, r1 = rg.y;
  T acc = T(0), dii = T(1);
  if (TRSV && mine) {
    acc = static_cast<const T*>(a.B)[row];
    dii = ld_stream(val + r1);
  }
  acc = stream_accumulate<T, TRSV, VEC, false>(nr, r0, r1 - r0, acc, TRSV ? a.Lci : a.Aci, nullptr, val, X,
                                               lane, w, a.ls, tr);
  if (mine) {
    if constexpr (TRSV) st_co(X + row, publishable(acc / dii));
    else __builtin_nontemporal_store(acc, static_cast<T*>(a.Y) + row);
  }
  if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
}

// Coarsened SpTRSV item (rows on several local wavefronts, sorted by local
// wavefront): dev::chunk_solve (stream.h) over the rows' off-diagonals.
template <typename T>
__device__ __forceinline__ void item_chunk(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w, T* xl,
                                           int it) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const T* __restrict__ val = static_cast<const T*>(a.Lv);
  unsigned long long* tr = trace_slots(a, it);
  if (tr && lane == 0) tr[0] = __builtin_amdgcn_s_memrealtime();
  const int row = mine ? a.order[q0 + lane] : 0;
  const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[q0 + lane] : make_int2(0, 0);
  const int r0 = rg.x, r1 = rg.y;  // off-diagonals; the diagonal sits at r1
  const int myloc = mine ? int(a.lloc[q0 + lane]) : 0;
  const int maxloc = int(a.lloc[q1 - 1]);
  const T acc = mine ? static_cast<const T*>(a.B)[row] : T(0);
  const T dii = mine ? ld_stream(val + r1) : T(1);
  dev::chunk_solve<T, false>(nr, r0, r1 - r0, myloc, maxloc, acc, dii, a.Lci, nullptr, val, a.eloc,
                             static_cast<T*>(a.X), row, lane, w, xl, a.ls, tr);
  if (tr && lane == 0) tr[3] = __builtin_amdgcn_s_memrealtime();
}

// The next ticket is claimed before the current item is processed, so the
// claim's round trip overlaps the item's loads.  Deadlock freedom still
// holds: a wave's prefetched ticket is larger than the item it works on, so
// the smallest claimed-but-unfinished item is always one being processed.
// With a coarsened plan (a.lloc != nullptr) SpTRSV items whose rows span
// several local wavefronts run through item_chunk.
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void k_ts_fused(TsArgs a) {
  __shared__ WaveLds<T> lds[kWaves];
  __shared__ T xloc[kWaves][65];  // item-local x by slot; [64] = 1.0 (see chunk_steps)
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[threadIdx.x >> 6];
  T* xl = xloc[threadIdx.x >> 6];
  if (lane == 0) xl[64] = T(1);
  dev::reset_next_launch(a.ls);
  int t = dev::claim(a.ls, lane);
  while (t < a.n_work) {
    const int tn = dev::claim(a.ls, lane);
    const int it = a.item_list ? a.item_list[t] : t;
    const int q0 = a.item_ptr[it], q1 = a.item_ptr[it + 1];
    if (a.order[q0] < a.n) {
      if (a.lloc && a.lloc[q1 - 1] != 0) item_chunk<T>(a, q0, q1, lane, w, xl, it);
      else item_stream<T, true, 2>(a, q0, q1, lane, w, it);
    } else {
      item_stream<T, false, 2>(a, q0, q1, lane, w, it);
    }
    t = tn;
  }
}

// ---------------------------------------------- kernel combinations 1, 2 --
// Table 2, combination 2: y = A x, z = L^{-1} y, and combination 1:
// x = L^{-1} b, z = L^{-1} x.  In both the second kernel's row i needs only
// row i of the first (F = I), so the item of SpTRSV row i computes both
// (the paper's interleaved packing): row i of the product, or the first
// solve's x_i, then z_i.  The SpTRSV plan (level or coarsened items) is the
// one of the fused executor; every sum runs in the definition's order.

// One triangular solve of an item's rows from the starting values acc;
// publishes into out and returns the lane's own result.
template <typename T>
__device__ __forceinline__ T solve_rows(const TsArgs& a, int q0, int q1, int lane, WaveLds<T>& w, T* xl, int row,
                                        int r0, int r1, T acc, T dii, T* out) {
  const int nr = q1 - q0;
  const bool mine = lane < nr;
  const T* __restrict__ val = static_cast<const T*>(a.Lv);
  if (a.lloc && a.lloc[q1 - 1] != 0) {
    const int myloc = mine ? int(a.lloc[q0 + lane]) : 0;
    return dev::chunk_solve<T, false>(nr, r0, r1 - r0, myloc, int(a.lloc[q1 - 1]), acc, dii, a.Lci, nullptr, val,
                                      a.eloc, out, row, lane, w, xl, a.ls, nullptr);
  }
  acc = stream_accumulate<T, true, 2, false>(nr, r0, r1 - r0, acc, a.Lci, nullptr, val, out, lane, w, a.ls);
  const T v = publishable(acc / dii);
  if (mine) st_co(out + row, v);
  return v;
}

// MODE 2: B = x (input), Y = y (optional output), X = z.
// MODE 1: B = b, X = x, Y = z.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlockThreads) void k_pair(TsArgs a) {
  __shared__ WaveLds<T> lds[kWaves];
  __shared__ T xloc[kWaves][65];  // item-local results by slot; [64] = 1.0
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[threadIdx.x >> 6];
  T* xl = xloc[threadIdx.x >> 6];
  if (lane == 0) xl[64] = T(1);
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ B = static_cast<const T*>(a.B);
  dev::reset_next_launch(a.ls);
  int t = dev::claim(a.ls, lane);
  while (t < a.n_work) {
    const int tn = dev::claim(a.ls, lane);
    const int it = a.item_list[t];
    const int q0 = a.item_ptr[it], q1 = a.item_ptr[it + 1];
    const bool mine = lane < q1 - q0;
    const int row = mine ? a.order[q0 + lane] : 0;
    const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[q0 + lane] : make_int2(0, 0);
    const T dii = mine ? ld_stream(Lv + rg.y) : T(1);
    if constexpr (MODE == 2) {
      const int p0 = mine ? a.Arp[row] : 0, p1 = mine ? a.Arp[row + 1] : 0;
      const T yi = stream_accumulate<T, false, 0, false>(q1 - q0, p0, p1 - p0, T(0), a.Aci, nullptr,
                                                         static_cast<const T*>(a.Av), B, lane, w, a.ls);
      if (mine && a.Y) __builtin_nontemporal_store(yi, static_cast<T*>(a.Y) + row);
      solve_rows<T>(a, q0, q1, lane, w, xl, row, rg.x, rg.y, yi, dii, static_cast<T*>(a.X));
    } else {
      const T bi = mine ? B[row] : T(0);
      const T xi = solve_rows<T>(a, q0, q1, lane, w, xl, row, rg.x, rg.y, bi, dii, static_cast<T*>(a.X));
      solve_rows<T>(a, q0, q1, lane, w, xl, row, rg.x, rg.y, xi, dii, static_cast<T*>(a.Y));
    }
    t = tn;
  }
}

// ------------------------------------------------------------- k > 1 ------
// KB lanes per row, one lane per right-hand side of the block; 64/KB rows
// at a time (the multi-RHS plan cuts items to that many rows).  B, the
// solution xi (filled with the pending pattern before the launch) and Y are
// in the interleaved block layout: row j of block b holds its KB values
// contiguously at [(b * rows + j) * KB], so a lane's gather of x_j and its
// reads and writes of row i are coalesced across the row's lanes.  Work
// index t = item * nblk + block.  Each lane runs its row's entries in
// ascending order (b_i minus each rounded product), kU entries at a time:
// their indices and values, then their x, are loaded together.  Load modes:
// kPoll (fused executor) waits for the pending x of the whole wavefront
// together (dev::wait_ptrs); kCoherent (level set: x written in this launch
// before a grid barrier) reads device-coherent values without waiting;
// kFinal (a later launch) reads through the caches.
constexpr int kU = 8;
enum LoadMode { kPoll, kCoherent, kFinal };

template <typename T, int KB, bool TRSV, LoadMode MODE>
__device__ __forceinline__ T row_multi(const int32_t* __restrict__ col, const T* __restrict__ val, const T* xi,
                                       int p0, int p1, int c, T acc, int lane, const LaunchState& ls) {
  int nch = (p1 - p0 + kU - 1) / kU;
  if constexpr (MODE == kPoll) {  // the wait is wave-wide: every lane runs the same number of rounds
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) nch = max(nch, __shfl_xor(nch, d, 64));
  }
  for (int ch = 0; ch < nch; ++ch) {
    const int c0 = p0 + ch * kU;
    int j[kU];
    T v[kU], xv[kU];
    const T* ptr[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int p = c0 + u;
      const bool h = p < p1;
      j[u] = h ? col[p] : -1;
      v[u] = h ? val[p] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      ptr[u] = j[u] >= 0 ? xi + size_t(j[u]) * KB + c : nullptr;
      if constexpr (MODE == kFinal) xv[u] = ptr[u] ? *ptr[u] : T(0);
      else xv[u] = ptr[u] ? ld_co(ptr[u]) : T(0);
    }
    if constexpr (MODE == kPoll) dev::wait_ptrs<T, kU>(ptr, xv, lane, ls);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (j[u] < 0) break;
      const T pr = v[u] * xv[u];
      if constexpr (TRSV) acc = acc - pr;
      else acc = acc + pr;
    }
  }
  return acc;
}

template <typename T, int KB, LoadMode MODE>
__device__ __forceinline__ void trsv_rows_multi(const TsArgs& a, int q0, int q1, int blk, int lane) {
  constexpr int RPB = 64 / KB;
  const int c = lane % KB;
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const size_t boff = size_t(blk) * size_t(a.n) * KB;
  const T* __restrict__ B = static_cast<const T*>(a.B) + boff;
  T* xi = static_cast<T*>(a.xi) + boff;
  for (int base = q0; base < q1; base += RPB) {
    const int q = base + lane / KB;
    const bool act = q < q1;
    const int i = act ? a.order[q] : 0;
    const int r0 = act ? a.Lrp[i] : 0;
    const int rd = act ? a.Lrp[i + 1] - 1 : 0;
    const T bi = act ? B[size_t(i) * KB + c] : T(0);
    const T dii = act ? Lv[rd] : T(1);
    const T s = row_multi<T, KB, true, MODE>(a.Lci, Lv, xi, r0, rd, c, bi, lane, a.ls);
    if (act) st_co(xi + size_t(i) * KB + c, publishable(s / dii));
  }
}

template <typename T, int KB>
__device__ __forceinline__ void spmv_rows_multi(const TsArgs& a, int q0, int q1, int blk, int lane) {
  constexpr int RPB = 64 / KB;
  const int c = lane % KB;
  const T* __restrict__ Av = static_cast<const T*>(a.Av);
  T* __restrict__ Y = static_cast<T*>(a.Y) + size_t(blk) * size_t(a.m) * KB;
  const T* xi = static_cast<const T*>(a.xi) + size_t(blk) * size_t(a.n) * KB;
  for (int base = q0; base < q1; base += RPB) {
    const int q = base + lane / KB;
    const bool act = q < q1;
    const int r = act ? a.order[q] - a.n : 0;
    const int p0 = act ? a.Arp[r] : 0;
    const int p1 = act ? a.Arp[r + 1] : 0;
    const T s = row_multi<T, KB, false, kPoll>(a.Aci, Av, xi, p0, p1, c, T(0), lane, a.ls);
    if (act) __builtin_nontemporal_store(s, Y + size_t(r) * KB + c);
  }
}

template <typename T, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_ts_multi(TsArgs a) {
  const int lane = threadIdx.x & 63;
  dev::reset_next_launch(a.ls);
  const int total = a.n_work * a.nblk;
  int t = dev::claim(a.ls, lane);
  while (t < total) {
    const int tn = dev::claim(a.ls, lane);
    const int w = t / a.nblk;
    const int blk = t - w * a.nblk;
    const int it = a.item_list ? a.item_list[w] : w;
    const int q0 = a.item_ptr[it], q1 = a.item_ptr[it + 1];
    if (a.order[q0] < a.n) trsv_rows_multi<T, KB, kPoll>(a, q0, q1, blk, lane);
    else spmv_rows_multi<T, KB>(a, q0, q1, blk, lane);
    t = tn;
  }
}

// Fill a solution buffer with the pending pattern before a launch.
template <typename T>
__global__ void k_fill_pending(T* p, size_t count) {
  const T v = __builtin_bit_cast(T, dev::Pending<T>::bits);
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < count; k += size_t(gridDim.x) * blockDim.x)
    p[k] = v;
}

// ---------------------------------------------------------- level set ----
// Unfused baseline, same per-item arithmetic: the SpTRSV items of one level
// are spread over all wavefronts of a cooperative grid, then a grid-wide
// barrier (no readiness protocol); afterwards a separate launch runs the
// SpMV items.  x is read and written with device-coherent accesses so the
// barrier only has to wait for stores to complete (dev::grid_barrier).
template <typename T, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_trsv_levelset(LevelArgs la) {
  __shared__ WaveLds<T> lds[KB == 1 ? kWaves : 1];
  const TsArgs& a = la.ts;
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[KB == 1 ? (threadIdx.x >> 6) : 0];
  dev::reset_next_launch(a.ls);
  const int wave = int(blockIdx.x) * kWaves + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * kWaves;
  int32_t gen = 0;
  for (int lv = 0; lv < la.depth; ++lv) {
    const int t0 = la.lvl_item_ptr[lv], t1 = la.lvl_item_ptr[lv + 1];
    for (int t = t0 + wave; t < t1; t += nwaves) {
      const int it = a.item_list[t];
      const int q0 = a.item_ptr[it], q1 = a.item_ptr[it + 1];
      if constexpr (KB == 1) item_stream<T, true, 1>(a, q0, q1, lane, w);
      else for (int blk = 0; blk < a.nblk; ++blk) trsv_rows_multi<T, KB, kCoherent>(a, q0, q1, blk, lane);
    }
    if (lv + 1 < la.depth) dev::grid_barrier(a.ls, gen);
  }
}

// SpMV items (all inputs final), grid-stride over the item list.
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void k_spmv_items(TsArgs a) {
  __shared__ WaveLds<T> lds[kWaves];
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[threadIdx.x >> 6];
  const int wave = int(blockIdx.x) * kWaves + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * kWaves;
  for (int t = wave; t < a.n_work; t += nwaves) {
    const int it = a.item_list[t];
    item_stream<T, false, 0>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, w);
  }
}

// Plain CSR SpMV over interleaved blocks (multi-RHS baseline): KB lanes per
// row, one per right-hand side, 64 / KB rows per wavefront, ascending
// entries; x is final (written by an earlier launch).
template <typename T, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_spmv_multi(SpmvArgs a) {
  constexpr int RPB = 64 / KB;
  const int lane = threadIdx.x & 63;
  const int c = lane % KB;
  const int wave = int(blockIdx.x) * kWaves + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * kWaves;
  const int groups = (a.m + RPB - 1) / RPB;
  const T* __restrict__ Av = static_cast<const T*>(a.Av);
  for (int u = wave; u < groups * a.nblk; u += nwaves) {
    const int blk = u % a.nblk;
    const int r = (u / a.nblk) * RPB + lane / KB;
    const T* X = static_cast<const T*>(a.X) + size_t(blk) * size_t(a.n) * KB;
    T* Y = static_cast<T*>(a.Y) + size_t(blk) * size_t(a.m) * KB;
    const bool act = r < a.m;
    const int p0 = act ? a.Arp[r] : 0, p1 = act ? a.Arp[r + 1] : 0;
    const T s = row_multi<T, KB, false, kFinal>(a.Aci, Av, X, p0, p1, c, T(0), lane, LaunchState{});
    if (act) __builtin_nontemporal_store(s, Y + size_t(r) * KB + c);
  }
}

template <typename T>
hipError_t levelset_launch(const LevelArgs& a, int grid, hipStream_t st) {
  void* args[] = {const_cast<LevelArgs*>(&a)};
#define SF_LS(KB)                                                                                          \
  if (a.ts.kb == KB)                                                                                       \
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_trsv_levelset<T, KB>), dim3(grid), \
                                      dim3(kBlockThreads), args, 0, st);
  SF_LS(1) SF_LS(2) SF_LS(4) SF_LS(8) SF_LS(16) SF_LS(32) SF_LS(64)
#undef SF_LS
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t ts_multi_dispatch(const TsArgs& a, int kb, int grid, hipStream_t st) {
#define SF_TM(KB)                                                                    \
  if (kb == KB) {                                                                    \
    hipLaunchKernelGGL((k_ts_multi<T, KB>), dim3(grid), dim3(kBlockThreads), 0, st, a); \
    return hipGetLastError();                                                        \
  }
  SF_TM(2) SF_TM(4) SF_TM(8) SF_TM(16) SF_TM(32) SF_TM(64)
#undef SF_TM
  return hipErrorInvalidValue;
}

template <typename K>
int occ(K kernel) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel),
                                                   kBlockThreads, 0) != hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

int cu_count() {
  int dev = 0, cus = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  return cus;
}

}  // namespace

hipError_t launch_ts_fused(const TsArgs& a, int dtype, int grid, hipStream_t st) {
  if (!a.qrng || !a.order || !a.item_ptr) return hipErrorInvalidValue;  // rows are streamed by claim position
  if (dtype == 0) hipLaunchKernelGGL(k_ts_fused<double>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  else hipLaunchKernelGGL(k_ts_fused<float>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_pair(const TsArgs& a, int dtype, int mode, int grid, hipStream_t st) {
  if (!a.qrng || !a.order || !a.item_ptr || !a.item_list) return hipErrorInvalidValue;
  if (mode == 2) {
    if (dtype == 0) hipLaunchKernelGGL((k_pair<double, 2>), dim3(grid), dim3(kBlockThreads), 0, st, a);
    else hipLaunchKernelGGL((k_pair<float, 2>), dim3(grid), dim3(kBlockThreads), 0, st, a);
  } else {
    if (dtype == 0) hipLaunchKernelGGL((k_pair<double, 1>), dim3(grid), dim3(kBlockThreads), 0, st, a);
    else hipLaunchKernelGGL((k_pair<float, 1>), dim3(grid), dim3(kBlockThreads), 0, st, a);
  }
  return hipGetLastError();
}
int occupancy_pair(int dtype, int mode) {
  if (mode == 2) return dtype == 0 ? occ(k_pair<double, 2>) : occ(k_pair<float, 2>);
  return dtype == 0 ? occ(k_pair<double, 1>) : occ(k_pair<float, 1>);
}
hipError_t launch_ts_multi(const TsArgs& a, int dtype, int kb, int grid, hipStream_t st) {
  if (!a.order || !a.item_ptr || !a.xi || !a.B || a.nblk < 1 || (a.Y && !a.Arp)) return hipErrorInvalidValue;
  return dtype == 0 ? ts_multi_dispatch<double>(a, kb, grid, st) : ts_multi_dispatch<float>(a, kb, grid, st);
}
hipError_t launch_trsv_levelset(const LevelArgs& a, int dtype, int grid, hipStream_t st) {
  if (!a.ts.order || !a.ts.item_ptr || !a.ts.item_list || !a.lvl_item_ptr) return hipErrorInvalidValue;
  if (a.ts.kb == 1 ? !a.ts.qrng : (!a.ts.xi || a.ts.nblk < 1)) return hipErrorInvalidValue;
  return dtype == 0 ? levelset_launch<double>(a, grid, st) : levelset_launch<float>(a, grid, st);
}
hipError_t launch_spmv_items(const TsArgs& a, int dtype, hipStream_t st) {
  if (!a.qrng || !a.order || !a.item_ptr || !a.item_list) return hipErrorInvalidValue;
  const int grid = cu_count() * 8;
  if (dtype == 0) hipLaunchKernelGGL(k_spmv_items<double>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  else hipLaunchKernelGGL(k_spmv_items<float>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}
template <typename T>
hipError_t spmv_multi_dispatch(const SpmvArgs& a, int grid, hipStream_t st) {
#define SF_SM(KB)                                                                      \
  if (a.kb == KB) {                                                                    \
    hipLaunchKernelGGL((k_spmv_multi<T, KB>), dim3(grid), dim3(kBlockThreads), 0, st, a); \
    return hipGetLastError();                                                          \
  }
  SF_SM(2) SF_SM(4) SF_SM(8) SF_SM(16) SF_SM(32) SF_SM(64)
#undef SF_SM
  return hipErrorInvalidValue;
}
hipError_t launch_spmv(const SpmvArgs& a, int dtype, hipStream_t st) {
  if (a.m <= 0) return hipSuccess;
  if (!a.Arp || !a.Aci || !a.Av || !a.X || !a.Y || a.kb < 2 || a.nblk < 1) return hipErrorInvalidValue;
  const long units = long((a.m + 64 / a.kb - 1) / (64 / a.kb)) * a.nblk;
  long grid = (units + kWaves - 1) / kWaves;
  grid = grid < 1 ? 1 : (grid > cu_count() * 32 ? cu_count() * 32 : grid);
  return dtype == 0 ? spmv_multi_dispatch<double>(a, int(grid), st) : spmv_multi_dispatch<float>(a, int(grid), st);
}
hipError_t launch_fill_pending(void* p, size_t count, int dtype, hipStream_t st) {
  if (count == 0) return hipSuccess;
  size_t g = (count + 255) / 256;
  const int grid = int(g > 16384 ? 16384 : g);
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill_pending<double>, dim3(grid), dim3(256), 0, st, static_cast<double*>(p), count);
  else
    hipLaunchKernelGGL(k_fill_pending<float>, dim3(grid), dim3(256), 0, st, static_cast<float*>(p), count);
  return hipGetLastError();
}
int occupancy_ts_fused(int dtype) {
  return dtype == 0 ? occ(k_ts_fused<double>) : occ(k_ts_fused<float>);
}
int occupancy_ts_multi(int dtype, int kb) {
  (void)kb;
  return dtype == 0 ? occ(k_ts_multi<double, 8>) : occ(k_ts_multi<float, 8>);
}
int occupancy_trsv_levelset(int dtype, int kb) {
  if (kb > 1) return dtype == 0 ? occ(k_trsv_levelset<double, 8>) : occ(k_trsv_levelset<float, 8>);
  return dtype == 0 ? occ(k_trsv_levelset<double, 1>) : occ(k_trsv_levelset<float, 1>);
}

}  // namespace sf
