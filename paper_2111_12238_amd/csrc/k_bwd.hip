// Backward executor: the adjoint of y = A L^{-1} b in one persistent launch.
//
// With g = dloss/dy, the gradients are lambda = L^{-T} (A^T g), grad_b =
// lambda and grad_L = -(lambda x^T) on the pattern of L.  The transposed
// solve runs over its own schedule (reversed wavefronts of L^T).  Row i of
// the upper solve
//   1. computes c_i = sum_r A_ri g_r over row i of A^T (ascending r; it
//      depends on nothing: the paper's SpMV -> SpTRSV pair with the product
//      interleaved into the solve),
//   2. subtracts L_ji lambda_j for j > i in ascending j, each lambda_j
//      observed through the value-as-flag protocol (grad_B is filled with the
//      pending pattern before the launch and is the lambda buffer),
//   3. divides by L_ii and publishes lambda_i (coarsened items resolve
//      their own rows' lambda values in LDS, dev::chunk_solve),
//   4. writes grad_L[p] = -lambda_i x_k for every stored L_ik of row i of L
//      (x is final input data).
// The arithmetic is the sequential definition's, term by term, so FP64
// gradients are bit-identical to the oracle's.  Values of L^T and A^T are
// read through the inspector's transpose maps; grad_L is written in the CSR
// order of L.
#pragma clang fp contract(off)

#include "region_core.h"

namespace sf {
namespace {

using dev::kWaves;
using dev::publishable;
using dev::st_co;
using dev::stream_accumulate;
using dev::WaveLds;

// grad_L[p] = -lambda_i x_j for every stored (i, j) of the item's rows i of
// L: the rows' entries are concatenated and dealt to the lanes, kRounds per
// lane and pass (as the entry stream deals a solve's terms), each row's lane
// laying out its positions and its lambda_i in LDS, so one round of loads
// serves every entry and consecutive lanes store consecutive entries.
template <typename T>
__device__ __forceinline__ void grad_rows(const int32_t* __restrict__ Lrp, const int32_t* __restrict__ Lci,
                                          const T* __restrict__ X, T* __restrict__ gL, int nr, int i, T li, int lane,
                                          WaveLds<T>& w) {
  using dev::kPass;
  using dev::kRounds;
  const bool mine = lane < nr;
  const int r0 = mine ? Lrp[i] : 0;
  const int len = mine ? Lrp[i + 1] - r0 : 0;
  int incl = len;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(incl, d, 64);
    if (lane >= d) incl += t;
  }
  const int off = incl - len;
  const int total = __shfl(incl, 63, 64);
  const T nli = -li;
  for (int base = 0; base < total; base += kPass) {
    __builtin_amdgcn_wave_barrier();
    if (mine) {
      const int lo = max(off, base), hi = min(off + len, base + kPass);
      for (int t = lo; t < hi; ++t) {
        w.pos[t - base] = r0 + (t - off);
        w.prod[t - base] = nli;
      }
    }
    __builtin_amdgcn_wave_barrier();
    int p[kRounds];
    T f[kRounds], xv[kRounds];
#pragma unroll
    for (int e = 0; e < kRounds; ++e) {
      const int k = base + lane + 64 * e;
      p[e] = k < total ? w.pos[k - base] : -1;
      f[e] = k < total ? w.prod[k - base] : T(0);
    }
#pragma unroll
    for (int e = 0; e < kRounds; ++e) xv[e] = p[e] >= 0 ? X[Lci[p[e]]] : T(0);
#pragma unroll
    for (int e = 0; e < kRounds; ++e)
      if (p[e] >= 0) __builtin_nontemporal_store(f[e] * xv[e], gL + p[e]);
  }
  __builtin_amdgcn_wave_barrier();
}

// With a coarsened plan (a.lloc != nullptr), items whose rows span several
// local wavefronts solve their lambda values through dev::chunk_solve.
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void k_bwd(BwdArgs a) {
  __shared__ WaveLds<T> lds[kWaves];
  __shared__ T lloc_x[kWaves][65];  // item-local lambda by slot; [64] = 1.0
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[threadIdx.x >> 6];
  T* xl = lloc_x[threadIdx.x >> 6];
  if (lane == 0) xl[64] = T(1);
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ Av = static_cast<const T*>(a.Av);
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const T* __restrict__ Gv = static_cast<const T*>(a.G);
  T* lam = static_cast<T*>(a.lam);
  T* __restrict__ gL = static_cast<T*>(a.gradL);
  dev::reset_next_launch(a.ls);
  int t = dev::claim(a.ls, lane);
  while (t < a.n_work) {
    const int tn = dev::claim(a.ls, lane);
    const int q0 = a.item_ptr[t], q1 = a.item_ptr[t + 1];
    const int nr = q1 - q0;
    const bool mine = lane < nr;
    const int i = mine ? a.order[q0 + lane] : 0;
    const int c0 = mine ? a.ATrp[i] : 0, c1 = mine ? a.ATrp[i + 1] : 0;
    const int e0 = mine ? a.LTrp[i] : 0, e1 = mine ? a.LTrp[i + 1] : 0;  // diagonal first
    const T lii = mine ? Lv[a.LTmap[e0]] : T(1);
    const T c = stream_accumulate<T, false, 0, true>(nr, c0, c1 - c0, T(0), a.ATci, a.ATmap, Av, Gv, lane, w,
                                                     a.ls);
    T li;
    if (a.lloc && a.lloc[q1 - 1] != 0) {
      const int myloc = mine ? int(a.lloc[q0 + lane]) : 0;
      li = dev::chunk_solve<T, true>(nr, e0 + 1, e1 - (e0 + 1), myloc, int(a.lloc[q1 - 1]), c, lii, a.LTci,
                                     a.LTmap, Lv, a.eloc, lam, i, lane, w, xl, a.ls, nullptr);
    } else {
      const T acc = stream_accumulate<T, true, 2, true>(nr, e0 + 1, e1 - (e0 + 1), c, a.LTci, a.LTmap, Lv, lam,
                                                        lane, w, a.ls);
      li = publishable(acc / lii);
      if (mine) st_co(lam + i, li);
    }
    grad_rows(a.Lrp, a.Lci, X, gL, nr, i, li, lane, w);
    t = tn;
  }
}

// The backward region plan: regions of the transposed solve on blocks of a
// computing and a polling wavefront (region_core.h).  A region row i stages
// c_i = sum_r A_ri g_r (ascending r, from 0: the product interleaved into the
// solve, as above) as its right-hand side and L's column i below the
// diagonal as its entries; lambda is published through the readiness
// protocol.  The grad_L rows follow every region in claim order, as items of
// up to kGradRows rows of L in row order (64 per wavefront and pass), each
// lambda_i read through the readiness protocol, so no region waits for them.
constexpr int kGradRows = 256;

template <typename T>
__global__ __launch_bounds__(kRegionThreads) void k_bwd_region(BwdArgs a, RegionArgs r) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int32_t ticket;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ Av = static_cast<const T*>(a.Av);
  const T* __restrict__ Gv = static_cast<const T*>(a.G);
  const T* __restrict__ X = static_cast<const T*>(a.X);
  T* lam = static_cast<T*>(a.lam);
  T* __restrict__ gL = static_cast<T*>(a.gradL);
  const int R = r.rows_max;
  const int total = a.n_work + (a.n + kGradRows - 1) / kGradRows;
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
    if (t < a.n_work) {
      const int q0 = a.item_ptr[t], q1 = a.item_ptr[t + 1];
      auto stage = [&](const RegionLds<T>& L, int k) {
        const int i = a.order[q0 + k];
        const int e0 = a.LTrp[i], e1 = a.LTrp[i + 1];  // diagonal first
        // c_i: the row of A^T, eight entries' loads at a time, folded in order from 0
        T c = T(0);
        const int c0 = a.ATrp[i], c1 = a.ATrp[i + 1];
        for (int p0 = c0; p0 < c1; p0 += 8) {
          int mp[8], cp[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int p = min(p0 + e, c1 - 1);
            mp[e] = a.ATmap[p];
            cp[e] = a.ATci[p];
          }
          T av[8], gv[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            av[e] = Av[mp[e]];
            gv[e] = Gv[cp[e]];
          }
#pragma unroll
          for (int e = 0; e < 8; ++e)
            if (p0 + e < c1) c = c + av[e] * gv[e];
        }
        stage_row<T>(L, R, k, i, c, Lv[a.LTmap[e0]], r.roff[q0 + k], e1 - e0 - 1, Lv, a.LTmap, e0 + 1, r.code);
      };
      region_core<T>(r, t, q0, q1, r.batch_ptr[t], r.batch_ptr[t + 1], lds, nullptr, lam, a.ls, nullptr, stage);
    } else {
      // grad_L rows [g0, g1) of L: lambda_i through the readiness protocol
      const int g0 = (t - a.n_work) * kGradRows, g1 = min(a.n, g0 + kGradRows);
      auto* w = reinterpret_cast<WaveLds<T>*>(lds) + wid;
      for (int s0 = g0 + 64 * wid; s0 < g1; s0 += 128) {
        const int nr = min(64, g1 - s0);
        const bool mine = lane < nr;
        const int i = mine ? s0 + lane : 0;
        T li = mine ? dev::ld_co(lam + i) : T(0);
        int32_t spins = 0;
        while (__ballot(mine && dev::is_pending(li)) != 0) {
          if (mine && dev::is_pending(li)) li = dev::ld_co(lam + i);
          if (!dev::all_poll_round(spins, a.ls)) break;
        }
        grad_rows(a.Lrp, a.Lci, X, gL, nr, i, li, lane, *w);
      }
    }
    __syncthreads();
    if (wid == 0) {
      const int tn = dev::claim_ticket(a.ls, next_raw);
      if (lane == 0) ticket = tn;
    }
    __syncthreads();
  }
}

// Preconditioner apply, z = L^{-T} (L^{-1} r), the solve pair a PCG
// iteration with an incomplete Cholesky factor needs.  Work tickets
// [0, n_fwd) are the forward plan's SpTRSV items (w_i = (r_i - sum L_ij w_j)
// / L_ii), tickets [n_fwd, n_fwd + n_bwd) the transposed plan's items
// (z_i = (w_i - sum_{j>i} L_ji z_j) / L_ii, ascending j); a backward row
// reads its own w_i through the readiness protocol (F = I).  Every backward
// item follows every forward item in the claim order, so the order stays
// topological; with only backward tickets (n_fwd = 0, w final) the same
// kernel is the second launch of the unfused baseline.
template <typename T>
__global__ __launch_bounds__(kBlockThreads) void k_precond(PrecondArgs a) {
  __shared__ WaveLds<T> lds[kWaves];
  __shared__ T lloc_x[kWaves][65];  // item-local results by slot; [64] = 1.0
  const int lane = threadIdx.x & 63;
  WaveLds<T>& w = lds[threadIdx.x >> 6];
  T* xl = lloc_x[threadIdx.x >> 6];
  if (lane == 0) xl[64] = T(1);
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  T* W = static_cast<T*>(a.W);
  T* Z = static_cast<T*>(a.Z);
  dev::reset_next_launch(a.ls);
  int t = dev::claim(a.ls, lane);
  while (t < a.n_fwd + a.n_bwd) {
    const int tn = dev::claim(a.ls, lane);
    if (t < a.n_fwd) {
      const int it = a.fitems[t];
      const int q0 = a.fitem_ptr[it], q1 = a.fitem_ptr[it + 1], nr = q1 - q0;
      const bool mine = lane < nr;
      const int row = mine ? a.forder[q0 + lane] : 0;
      const int2 rg = mine ? reinterpret_cast<const int2*>(a.fqrng)[q0 + lane] : make_int2(0, 0);
      const T ri = mine ? static_cast<const T*>(a.R)[row] : T(0);
      const T dii = mine ? Lv[rg.y] : T(1);
      if (a.flloc && a.flloc[q1 - 1] != 0) {
        const int myloc = mine ? int(a.flloc[q0 + lane]) : 0;
        dev::chunk_solve<T, false>(nr, rg.x, rg.y - rg.x, myloc, int(a.flloc[q1 - 1]), ri, dii, a.Lci, nullptr, Lv,
                                   a.feloc, W, row, lane, w, xl, a.ls, nullptr);
      } else {
        const T acc = stream_accumulate<T, true, 2, false>(nr, rg.x, rg.y - rg.x, ri, a.Lci, nullptr, Lv, W, lane,
                                                           w, a.ls);
        if (mine) st_co(W + row, publishable(acc / dii));
      }
    } else {
      const int it = t - a.n_fwd;
      const int q0 = a.bitem_ptr[it], q1 = a.bitem_ptr[it + 1], nr = q1 - q0;
      const bool mine = lane < nr;
      const int i = mine ? a.border[q0 + lane] : 0;
      const int e0 = mine ? a.LTrp[i] : 0, e1 = mine ? a.LTrp[i + 1] : 0;  // diagonal first
      const T lii = mine ? Lv[a.LTmap[e0]] : T(1);
      int j[1] = {mine ? i : -1};
      T wi[1] = {mine ? dev::ld_co(W + i) : T(0)};
      dev::wait_ready<T, 1>(W, j, wi, lane, a.ls);
      if (a.blloc && a.blloc[q1 - 1] != 0) {
        const int myloc = mine ? int(a.blloc[q0 + lane]) : 0;
        dev::chunk_solve<T, true>(nr, e0 + 1, e1 - (e0 + 1), myloc, int(a.blloc[q1 - 1]), wi[0], lii, a.LTci,
                                  a.LTmap, Lv, a.beloc, Z, i, lane, w, xl, a.ls, nullptr);
      } else {
        const T acc = stream_accumulate<T, true, 2, true>(nr, e0 + 1, e1 - (e0 + 1), wi[0], a.LTci, a.LTmap, Lv, Z,
                                                          lane, w, a.ls);
        if (mine) st_co(Z + i, publishable(acc / lii));
      }
    }
    t = tn;
  }
}

// Preconditioner apply z = L^{-T} (L^{-1} r) on the two region plans, one
// block of a computing and a polling wavefront per region (region_core).
// Tickets [0, n_fwd) are the forward solve's regions (fitems: their item
// indices in the forward region plan; right-hand side r_i, w published into
// W); tickets [n_fwd, n_fwd + n_bwd) are the transposed solve's regions over
// L^T (right-hand side w_i, read through the readiness protocol while the
// region is staged; z published into Z).  Every transposed region follows
// every forward one in claim order, so the staging waits only on forward
// regions that are already claimed.
template <typename T>
__global__ __launch_bounds__(kRegionThreads) void k_precond_region(PrecondArgs a, RegionArgs rf, RegionArgs rb) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int32_t ticket;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ Rv = static_cast<const T*>(a.R);
  T* W = static_cast<T*>(a.W);
  T* Z = static_cast<T*>(a.Z);
  const int total = a.n_fwd + a.n_bwd;
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
    if (t < a.n_fwd) {
      const int item = a.fitems[t];
      const int q0 = a.fitem_ptr[item], q1 = a.fitem_ptr[item + 1];
      auto stage = [&](const RegionLds<T>& L, int k) {
        const int id = a.forder[q0 + k];
        const int2 rg = reinterpret_cast<const int2*>(a.fqrng)[q0 + k];
        stage_row<T>(L, rf.rows_max, k, id, Rv[id], dev::ld_stream(Lv + rg.y), rf.roff[q0 + k], rg.y - rg.x, Lv,
                     nullptr, rg.x, rf.code);
      };
      region_core<T>(rf, item, q0, q1, rf.batch_ptr[item], rf.batch_ptr[item + 1], lds, nullptr, W, a.ls, nullptr,
                     stage);
    } else {
      const int it = t - a.n_fwd;
      const int q0 = a.bitem_ptr[it], q1 = a.bitem_ptr[it + 1];
      auto stage = [&](const RegionLds<T>& L, int k) {
        const int i = a.border[q0 + k];
        const int e0 = a.LTrp[i], e1 = a.LTrp[i + 1];  // diagonal first
        // w_i, published by the forward region of row i
        T wi = dev::ld_co(W + i);
        int32_t spins = 0;
        while (is_pending(wi)) {
          __builtin_amdgcn_s_sleep(1);
          wi = dev::ld_co(W + i);
          if (++spins >= a.ls.spin_limit) {
            dev::report_timeout(a.ls);
            break;
          }
        }
        stage_row<T>(L, rb.rows_max, k, i, wi, Lv[a.LTmap[e0]], rb.roff[q0 + k], e1 - e0 - 1, Lv, a.LTmap, e0 + 1,
                     rb.code);
      };
      region_core<T>(rb, it, q0, q1, rb.batch_ptr[it], rb.batch_ptr[it + 1], lds, nullptr, Z, a.ls, nullptr,
                     stage);
    }
    __syncthreads();
    if (wid == 0) {
      const int tn = dev::claim_ticket(a.ls, next_raw);
      if (lane == 0) ticket = tn;
    }
    __syncthreads();
  }
}

template <typename K>
int occ(K kernel) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel),
                                                   kBlockThreads, 0) != hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

hipError_t launch_bwd(const BwdArgs& a, int dtype, int g, int grid, hipStream_t st) {
  (void)g;
  if (dtype == 0) hipLaunchKernelGGL(k_bwd<double>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  else hipLaunchKernelGGL(k_bwd<float>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_precond(const PrecondArgs& a, int dtype, int grid, hipStream_t st) {
  if ((a.n_fwd > 0 && (!a.forder || !a.fqrng || !a.fitem_ptr || !a.fitems)) || !a.border || !a.bitem_ptr)
    return hipErrorInvalidValue;
  if (dtype == 0) hipLaunchKernelGGL(k_precond<double>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  else hipLaunchKernelGGL(k_precond<float>, dim3(grid), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}

int occupancy_precond(int dtype) { return dtype == 0 ? occ(k_precond<double>) : occ(k_precond<float>); }

size_t bwd_region_lds(const RegionArgs& r, int dtype) {
  const int vb = dtype == 0 ? 8 : 4;
  const size_t reg = region_lds_bytes(r.rows_max, r.entries_max, r.ext_max, r.batches_max, vb);
  const size_t sp = 2 * (dtype == 0 ? sizeof(WaveLds<double>) : sizeof(WaveLds<float>));
  return reg > sp ? reg : sp;
}
hipError_t launch_bwd_region(const BwdArgs& a, const RegionArgs& r, int dtype, int grid, hipStream_t st) {
  if (!a.order || !a.item_ptr || !r.batch || !r.batch_ptr || !r.ext_ptr || !r.roff || !r.code)
    return hipErrorInvalidValue;
  const size_t lds = bwd_region_lds(r, dtype);
  if (dtype == 0) hipLaunchKernelGGL(k_bwd_region<double>, dim3(grid), dim3(kRegionThreads), lds, st, a, r);
  else hipLaunchKernelGGL(k_bwd_region<float>, dim3(grid), dim3(kRegionThreads), lds, st, a, r);
  return hipGetLastError();
}
int occupancy_bwd_region(const RegionArgs& r, int dtype) {
  const size_t lds = bwd_region_lds(r, dtype);
  int b = 0;
  const void* k = dtype == 0 ? reinterpret_cast<const void*>(k_bwd_region<double>)
                             : reinterpret_cast<const void*>(k_bwd_region<float>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kRegionThreads, lds) != hipSuccess) return 1;
  return b < 1 ? 1 : b;
}

size_t precond_region_lds(const RegionArgs& rf, const RegionArgs& rb, int dtype) {
  const int vb = dtype == 0 ? 8 : 4;
  const size_t f = region_lds_bytes(rf.rows_max, rf.entries_max, rf.ext_max, rf.batches_max, vb);
  const size_t b = region_lds_bytes(rb.rows_max, rb.entries_max, rb.ext_max, rb.batches_max, vb);
  return f > b ? f : b;
}
hipError_t launch_precond_region(const PrecondArgs& a, const RegionArgs& rf, const RegionArgs& rb, int dtype,
                                 int grid, hipStream_t st) {
  if (!a.forder || !a.fqrng || !a.fitem_ptr || !a.fitems || !a.border || !a.bitem_ptr || !rf.batch ||
      !rf.batch_ptr || !rf.ext_ptr || !rf.roff || !rf.code || !rb.batch || !rb.batch_ptr || !rb.ext_ptr || !rb.roff ||
      !rb.code)
    return hipErrorInvalidValue;
  const size_t lds = precond_region_lds(rf, rb, dtype);
  if (dtype == 0) hipLaunchKernelGGL(k_precond_region<double>, dim3(grid), dim3(kRegionThreads), lds, st, a, rf, rb);
  else hipLaunchKernelGGL(k_precond_region<float>, dim3(grid), dim3(kRegionThreads), lds, st, a, rf, rb);
  return hipGetLastError();
}
int occupancy_precond_region(const RegionArgs& rf, const RegionArgs& rb, int dtype) {
  const size_t lds = precond_region_lds(rf, rb, dtype);
  int b = 0;
  const void* k = dtype == 0 ? reinterpret_cast<const void*>(k_precond_region<double>)
                             : reinterpret_cast<const void*>(k_precond_region<float>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kRegionThreads, lds) != hipSuccess) return 1;
  return b < 1 ? 1 : b;
}

int occupancy_bwd(int dtype, int g) {
  (void)g;
  return dtype == 0 ? occ(k_bwd<double>) : occ(k_bwd<float>);
}

}  // namespace sf
