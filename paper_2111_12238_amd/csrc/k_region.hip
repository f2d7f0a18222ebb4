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

#include "region_core.h"

namespace sf {
namespace {

// One region of the fused SpTRSV -> SpMV executor: rows of L (entries
// [qrng.x, qrng.y), diagonal at qrng.y), right-hand side B.
template <typename T>
__device__ void region_rows(const TsArgs& a, const RegionArgs& r, int item, int q0, int q1, int b0, int b1,
                            char* lds, unsigned long long* tr) {
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ B = static_cast<const T*>(a.B);
  const int R = r.rows_max;
  auto stage = [&](const RegionLds<T>& L, int k) {
    const int id = a.order[q0 + k];
    const int2 rg = reinterpret_cast<const int2*>(a.qrng)[q0 + k];
    stage_row<T>(L, R, k, id, B[id], dev::ld_stream(Lv + rg.y), r.roff[q0 + k], rg.y - rg.x, Lv, nullptr, rg.x,
                 r.code);
  };
  region_core<T>(r, item, q0, q1, b0, b1, lds, tr, static_cast<T*>(a.X), a.ls, a.rtrace, stage);
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

// Kernel combinations 2 and 1 (Table 2) on the region plan's SpTRSV
// regions (item_list, n_work regions).  MODE 2: y = A x, z = L^{-1} y -- a
// region row stages y_i = sum_j A_ij x_j (A's row in order, from 0; x is
// input) as its right-hand side, stores it to Y, and the regions publish z
// into X.  MODE 1: x = L^{-1} b, z = L^{-1} x -- tickets [0, n_work) solve
// x into X from B, tickets [n_work, 2 n_work) solve z into Y, a row staging
// its x_i (F = I) through the readiness protocol; every z region follows
// every x region in claim order.
template <typename T, int MODE>
__global__ __launch_bounds__(kRegionThreads) void k_pair_region(TsArgs a, RegionArgs r) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int32_t ticket;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ B = static_cast<const T*>(a.B);
  const int R = r.rows_max;
  const int total = MODE == 1 ? 2 * a.n_work : a.n_work;
  dev::reset_next_launch(a.ls);
  if (wid == 0) {
    const int t = dev::claim(a.ls, lane);
    if (lane == 0) ticket = t;
  }
  __syncthreads();
  for (;;) {
    const int t = ticket;
    __syncthreads();
    if (t >= total) break;
    int32_t next_raw = 0;
    if (wid == 0) next_raw = dev::claim_issue(a.ls, lane);
    const bool second = MODE == 1 && t >= a.n_work;
    const int item = a.item_list[second ? t - a.n_work : t];
    const int q0 = a.item_ptr[item], q1 = a.item_ptr[item + 1];
    T* out = static_cast<T*>(second ? a.Y : a.X);
    auto stage = [&](const RegionLds<T>& L, int k) {
      const int id = a.order[q0 + k];
      const int2 rg = reinterpret_cast<const int2*>(a.qrng)[q0 + k];
      T bi;
      if constexpr (MODE == 2) {
        bi = T(0);
        const int p0 = a.Arp[id], p1 = a.Arp[id + 1];
        const T* __restrict__ Av = static_cast<const T*>(a.Av);
        for (int c0 = p0; c0 < p1; c0 += 8) {
          int cj[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) cj[e] = a.Aci[min(c0 + e, p1 - 1)];
          T av[8], xv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            av[e] = dev::ld_stream(Av + min(c0 + e, p1 - 1));
            xv[e] = B[cj[e]];
          }
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (c0 + e < p1) bi = bi + av[e] * xv[e];
        }
        if (a.Y) __builtin_nontemporal_store(bi, static_cast<T*>(a.Y) + id);
      } else if (second) {
        // x_i, published by the first solve's region of row i
        const T* xp = static_cast<const T*>(a.X) + id;
        bi = ld_co(xp);
        int32_t spins = 0;
        while (is_pending(bi)) {
          __builtin_amdgcn_s_sleep(1);
          bi = ld_co(xp);
          if (++spins >= a.ls.spin_limit) {
            dev::report_timeout(a.ls);
            break;
          }
        }
      } else {
        bi = B[id];
      }
      stage_row<T>(L, R, k, id, bi, dev::ld_stream(Lv + rg.y), r.roff[q0 + k], rg.y - rg.x, Lv, nullptr, rg.x,
                   r.code);
    };
    region_core<T>(r, item, q0, q1, r.batch_ptr[item], r.batch_ptr[item + 1], lds, nullptr, out, a.ls, nullptr,
                   stage);
    __syncthreads();
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

hipError_t launch_pair_region(const TsArgs& a, const RegionArgs& r, int dtype, int mode, int grid, hipStream_t st) {
  if (!a.order || !a.qrng || !a.item_ptr || !a.item_list || !r.batch || !r.batch_ptr || !r.ext_ptr || !r.roff ||
      !r.code || (mode == 2 && (!a.Arp || !a.Aci)) || (mode == 1 && !a.Y))
    return hipErrorInvalidValue;
  const int vb = dtype == 0 ? 8 : 4;
  const size_t lds = region_lds_bytes(r.rows_max, r.entries_max, r.ext_max, r.batches_max, vb);
  if (mode == 2) {
    if (dtype == 0) hipLaunchKernelGGL((k_pair_region<double, 2>), dim3(grid), dim3(kRegionThreads), lds, st, a, r);
    else hipLaunchKernelGGL((k_pair_region<float, 2>), dim3(grid), dim3(kRegionThreads), lds, st, a, r);
  } else {
    if (dtype == 0) hipLaunchKernelGGL((k_pair_region<double, 1>), dim3(grid), dim3(kRegionThreads), lds, st, a, r);
    else hipLaunchKernelGGL((k_pair_region<float, 1>), dim3(grid), dim3(kRegionThreads), lds, st, a, r);
  }
  return hipGetLastError();
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
