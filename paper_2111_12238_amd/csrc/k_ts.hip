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

#include <type_traits>

#include "ts_items.h"

namespace sf {
namespace {

// Per item the wavefront runs one chain of dependent loads: the rows' ids,
// ranges and local wavefronts (together), the rows' entries, then the x
// values.  Around it:
// - the next ticket is claimed right after the row loads are issued and
//   waited for with them, so the claim's round trip overlaps theirs;
// - the next item's range is loaded as soon as its ticket is known, during
//   this item, so the next item starts with its row loads;
// - the item's kind (SpTRSV or SpMV rows) is read off its first row's id.
// Deadlock freedom still holds: a wave's prefetched ticket is larger than
// the item it works on, so the smallest claimed-but-unfinished item is
// always one being processed.  With a coarsened plan (a.lloc != nullptr)
// SpTRSV items whose rows span several local wavefronts run through
// item_chunk_rows.
template <typename T, bool PRE>
__global__ __launch_bounds__(kBlockThreads) void k_ts_fused(TsArgs a) {
  using W = std::conditional_t<PRE, dev::WaveLdsPre<T>, WaveLds<T>>;
  __shared__ W lds[kWaves];
  __shared__ T xloc[kWaves][65];  // item-local x by slot; [64] = 1.0 (see chunk_steps)
  const int lane = threadIdx.x & 63;
  W& w = lds[threadIdx.x >> 6];
  T* xl = xloc[threadIdx.x >> 6];
  if (lane == 0) xl[64] = T(1);
  dev::reset_next_launch(a.ls);
  // several right-hand sides as separate chains: ticket t is column t % nc of
  // item t / nc, so all columns of an item come before the next item and the
  // claim order stays topological
  const int nc = a.col_units > 1 ? a.col_units : 1;
  const int total = a.n_work * nc;
  int t = dev::claim(a.ls, lane);
  int it = 0, q0 = 0, q1 = 0;
  if (t < total) item_range(a, t / nc, it, q0, q1);
  while (t < total) {
    const int c = t - (t / nc) * nc;
    TsArgs ac = a;
    if (nc > 1) {
      ac.B = static_cast<const T*>(a.B) + size_t(c) * size_t(a.ldb);
      ac.X = static_cast<T*>(a.X) + size_t(c) * size_t(a.ldx);
      if (a.Y) ac.Y = static_cast<T*>(a.Y) + size_t(c) * size_t(a.ldy);
    }
    unsigned long long* tr = trace_slots(a, it);
    if (tr && lane == 0) {
      // an item without entries loads and waits for nothing: its "loaded"
      // and "ready" stamps stay at its start
      const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
      tr[0] = t0;
      tr[1] = t0;
      tr[2] = t0;
      atomicAdd(tr + 4, 1ull);
    }
    const bool mine = lane < q1 - q0;
    const int id = mine ? a.order[q0 + lane] : 0;
    const int2 rg = mine ? reinterpret_cast<const int2*>(a.qrng)[q0 + lane] : make_int2(0, 0);
    const int myloc = (a.lloc && mine) ? int(a.lloc[q0 + lane]) : 0;
    const int a0 = (PRE && mine) ? a.apre[q0 + lane] : -1;  // prefix fusion: the row's prefix in A
    // the item's last local wavefront, on lane 0 (a uniform load would be
    // waited for at once, to move it to a scalar register)
    const int lastloc = (a.lloc && lane == 0) ? int(a.lloc[q1 - 1]) : 0;
    // the next ticket's atomic goes out after the row loads (a wait for
    // anything issued before it would otherwise wait for it too) and is
    // waited for with them: an empty asm statement ties its result to the
    // row loads, so the conversion cannot be scheduled ahead of them
    const int32_t raw = dev::claim_issue(a.ls, lane);
    int32_t pending = raw;
    __asm__ volatile("" : "+v"(pending) : "v"(id), "v"(lastloc));
    const int tn = dev::claim_ticket(a.ls, pending);
    const int maxloc = __shfl(lastloc, 0, 64);
    int itn = 0, q0n = 0, q1n = 0;
    if (tn < total) item_range(a, tn / nc, itn, q0n, q1n);
    if constexpr (PRE) {
      // level items only (no coarsened items with prefix fusion)
      if (__shfl(id, 0, 64) < a.n) {
        if (a.cached & 2) item_stream_rows_pre<T, 3>(ac, q0, q1, lane, w, tr, id, rg, a0);
        else item_stream_rows_pre<T, 2>(ac, q0, q1, lane, w, tr, id, rg, a0);
      } else if (a.cached & 1) {
        item_spmv_rows_from<T, 3>(ac, q0, q1, lane, w, tr, id, rg);
      } else {
        item_spmv_rows_from<T, 2>(ac, q0, q1, lane, w, tr, id, rg);
      }
    } else if (__shfl(id, 0, 64) < a.n) {  // lane 0 holds the item's first row (an item has >= 1 row)
      if (maxloc != 0) item_chunk_rows<T>(ac, q0, q1, lane, w, xl, tr, id, rg, myloc, maxloc);
      else if (a.cached & 2) item_stream_rows<T, true, 3>(ac, q0, q1, lane, w, tr, id, rg);
      else item_stream_rows<T, true, 2>(ac, q0, q1, lane, w, tr, id, rg);
    } else if (a.cached & 1) {
      item_stream_rows<T, false, 3>(ac, q0, q1, lane, w, tr, id, rg);
    } else {
      item_stream_rows<T, false, 2>(ac, q0, q1, lane, w, tr, id, rg);
    }
    t = tn;
    it = itn;
    q0 = q0n;
    q1 = q1n;
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

// Work index t = unit * nblk + block.  The next ticket is claimed before
// the current unit runs and its range is loaded inside it (see unit_multi),
// so neither is a round trip on the next unit's chain; deadlock freedom is
// as in k_ts_fused.
template <typename T, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_ts_multi(TsArgs a) {
  __shared__ MultiLds<T, KB> lds[kWaves];
  const int lane = threadIdx.x & 63;
  MultiLds<T, KB>& w = lds[threadIdx.x >> 6];
  dev::reset_next_launch(a.ls);
  const int total = a.n_work * a.nblk;
  int t = dev::claim(a.ls, lane);
  int2 rg = t < total ? a.unit_rng[t / a.nblk] : make_int2(0, 0);
  while (t < total) {
    const int tn = dev::claim(a.ls, lane);
    int2 rgn;
    unit_multi<T, KB, true>(a, rg.x, rg.y, t % a.nblk, lane, w, tn < total ? tn / a.nblk : -1, &rgn);
    t = tn;
    rg = rgn;
  }
}

// Fill a solution buffer with the pending pattern before a launch.
template <typename T>
__global__ void k_fill_pending(T* p, size_t count) {
  const T v = __builtin_bit_cast(T, dev::Pending<T>::bits);
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < count; k += size_t(gridDim.x) * blockDim.x)
    p[k] = v;
}
template <typename T>
__global__ void k_fill_pending_cols(T* p, int32_t rows, int32_t ld, int32_t ncols) {
  const T v = __builtin_bit_cast(T, dev::Pending<T>::bits);
  const size_t count = size_t(rows) * size_t(ncols);
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < count; k += size_t(gridDim.x) * blockDim.x) {
    const size_t c = k / size_t(rows), i = k - c * size_t(rows);
    p[i + c * size_t(ld)] = v;
  }
}

// ---------------------------------------------------------- level set ----
// Unfused baseline, same per-row arithmetic: the SpTRSV items of one level
// (several right-hand sides: the level's units times the blocks) are spread
// over all wavefronts of a cooperative grid, then a grid-wide barrier (no
// readiness protocol); afterwards a separate launch runs the SpMV.  x is
// read and written with device-coherent accesses so the barrier only has to
// wait for stores to complete (dev::grid_barrier).
template <typename T, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_trsv_levelset(LevelArgs la) {
  // one right-hand side: level items through item_stream; several: the
  // level's units (la.lvl_item_ptr indexes a.unit_rng) times the blocks
  using Lds = std::conditional_t<KB == 1, WaveLds<T>, MultiLds<T, (KB > 1 ? KB : 2)>>;
  __shared__ Lds lds[kWaves];
  const TsArgs& a = la.ts;
  const int lane = threadIdx.x & 63;
  Lds& w = lds[threadIdx.x >> 6];
  dev::reset_next_launch(a.ls);
  const int wave = int(blockIdx.x) * kWaves + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * kWaves;
  int32_t gen = 0;
  for (int lv = 0; lv < la.depth; ++lv) {
    const int t0 = la.lvl_item_ptr[lv], t1 = la.lvl_item_ptr[lv + 1];
    if constexpr (KB == 1) {
      for (int t = t0 + wave; t < t1; t += nwaves) {
        const int it = a.item_list[t];
        item_stream<T, true, 1>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, w);
      }
    } else {
      for (int t = t0 * a.nblk + wave; t < t1 * a.nblk; t += nwaves) {
        const int2 rg = a.unit_rng[t / a.nblk];
        unit_multi<T, KB, false>(a, rg.x, rg.y, t % a.nblk, lane, w);
      }
    }
    if (lv + 1 < la.depth) dev::grid_barrier(a.ls, gen);
  }
}

// ------------------------------------------------------ static plans ----
// The paper's own schedule form (Sec. 3): a fused partitioning whose
// s-partitions are separated by a grid barrier and whose w-partitions each
// run on one wavefront, its rows in order (or the fused wavefront baseline,
// one s-partition per wavefront of the joint DAG).  x is read and written
// device-coherently, as in the level set; a wavefront waits for its own
// stores before the next batch of its w-partition, which may read them.
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void k_static(StaticArgs sa) {
  __shared__ WaveLds<T> lds[kWaves];
  const TsArgs& a = sa.ts;
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[threadIdx.x >> 6];
  dev::reset_next_launch(a.ls);
  const int wave = int(blockIdx.x) * kWaves + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * kWaves;
  int32_t gen = 0;
  for (int b = 0; b < sa.nb; ++b) {
    for (int wp = sa.s_ptr[b] + wave; wp < sa.s_ptr[b + 1]; wp += nwaves) {
      for (int bt = sa.w_batch[wp]; bt < sa.w_batch[wp + 1]; ++bt) {
        const int q0 = sa.batch_ptr[bt], q1 = sa.batch_ptr[bt + 1];
        if (a.order[q0] < a.n) item_stream<T, true, 1>(a, q0, q1, lane, w);
        else item_stream<T, false, 1>(a, q0, q1, lane, w);
        dev::stores_complete();
      }
    }
    if (b + 1 < sa.nb) dev::grid_barrier(a.ls, gen);
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
    const T s = row_final<T, KB>(a.Aci, Av, X, p0, p1, c);
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
  if (a.apre) {
    if (!a.Y || !a.Av || !a.Aci) return hipErrorInvalidValue;
    if (dtype == 0) hipLaunchKernelGGL((k_ts_fused<double, true>), dim3(grid), dim3(kBlockThreads), 0, st, a);
    else hipLaunchKernelGGL((k_ts_fused<float, true>), dim3(grid), dim3(kBlockThreads), 0, st, a);
  } else if (dtype == 0) {
    hipLaunchKernelGGL((k_ts_fused<double, false>), dim3(grid), dim3(kBlockThreads), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_ts_fused<float, false>), dim3(grid), dim3(kBlockThreads), 0, st, a);
  }
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
  if (!a.order || !a.qrng || !a.unit_rng || !a.xi || !a.B || a.nblk < 1 || (a.Y && !a.Arp))
    return hipErrorInvalidValue;
  return dtype == 0 ? ts_multi_dispatch<double>(a, kb, grid, st) : ts_multi_dispatch<float>(a, kb, grid, st);
}
hipError_t launch_trsv_levelset(const LevelArgs& a, int dtype, int grid, hipStream_t st) {
  if (!a.ts.order || !a.ts.qrng || !a.lvl_item_ptr) return hipErrorInvalidValue;
  if (a.ts.kb == 1 ? (!a.ts.item_ptr || !a.ts.item_list) : (!a.ts.unit_rng || !a.ts.xi || a.ts.nblk < 1))
    return hipErrorInvalidValue;
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
hipError_t launch_static(const StaticArgs& a, int dtype, int grid, hipStream_t st) {
  if (!a.ts.order || !a.ts.qrng || !a.s_ptr || !a.w_batch || !a.batch_ptr || a.nb < 0) return hipErrorInvalidValue;
  if (a.nb == 0) return hipSuccess;
  void* args[] = {const_cast<StaticArgs*>(&a)};
  const void* fn = dtype == 0 ? reinterpret_cast<const void*>(&k_static<double>)
                              : reinterpret_cast<const void*>(&k_static<float>);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlockThreads), args, 0, st);
}
int occupancy_static(int dtype) { return dtype == 0 ? occ(k_static<double>) : occ(k_static<float>); }
hipError_t launch_fill_pending_cols(void* p, int32_t rows, int32_t ld, int32_t ncols, int dtype, hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (!p || ld < rows) return hipErrorInvalidValue;
  size_t g = (size_t(rows) * size_t(ncols) + 255) / 256;
  const int grid = int(g > 16384 ? 16384 : g);
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill_pending_cols<double>, dim3(grid), dim3(256), 0, st, static_cast<double*>(p), rows, ld, ncols);
  else
    hipLaunchKernelGGL(k_fill_pending_cols<float>, dim3(grid), dim3(256), 0, st, static_cast<float*>(p), rows, ld, ncols);
  return hipGetLastError();
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
  return dtype == 0 ? occ(k_ts_fused<double, false>) : occ(k_ts_fused<float, false>);
}
int occupancy_ts_fused_pre(int dtype) {
  return dtype == 0 ? occ(k_ts_fused<double, true>) : occ(k_ts_fused<float, true>);
}
template <typename T>
int occ_multi(int kb, bool levelset) {
  switch (kb) {
    case 2: return levelset ? occ(k_trsv_levelset<T, 2>) : occ(k_ts_multi<T, 2>);
    case 4: return levelset ? occ(k_trsv_levelset<T, 4>) : occ(k_ts_multi<T, 4>);
    case 8: return levelset ? occ(k_trsv_levelset<T, 8>) : occ(k_ts_multi<T, 8>);
    case 16: return levelset ? occ(k_trsv_levelset<T, 16>) : occ(k_ts_multi<T, 16>);
    case 32: return levelset ? occ(k_trsv_levelset<T, 32>) : occ(k_ts_multi<T, 32>);
    default: return levelset ? occ(k_trsv_levelset<T, 64>) : occ(k_ts_multi<T, 64>);
  }
}
int occupancy_ts_multi(int dtype, int kb) { return dtype == 0 ? occ_multi<double>(kb, false) : occ_multi<float>(kb, false); }
int occupancy_trsv_levelset(int dtype, int kb) {
  if (kb > 1) return dtype == 0 ? occ_multi<double>(kb, true) : occ_multi<float>(kb, true);
  return dtype == 0 ? occ(k_trsv_levelset<double, 1>) : occ(k_trsv_levelset<float, 1>);
}

}  // namespace sf
