// Fused SpIC0 -> SpTRSV executor (FP64) and its level-set baseline.
//
// Row i of the zero fill-in incomplete Cholesky factor (Table 2, comb. 5),
// by the up-looking row recurrence, with P_i the stored columns of row i:
//     L_ij = (A_ij - sum_{k<j, k in P_i and P_j} L_ik L_jk) / L_jj,  j in P_i, j < i
//     L_ii = sqrt(A_ii - sum_{k<i} L_ik^2)
// and, in the same work item (the paper's interleaved packing: F = I, the
// solve of row i needs only the factor rows it already waited for),
//     x_i = (b_i - sum_{j<i} L_ij x_j) / L_ii.
// One flag per row covers both kernels: it is published once row i of L and
// x_i are stored.
//
// G lanes per row, lane t owns the t-th off-diagonal entry (rows with more
// than G off-diagonals are rejected by the caller).  The k-intersections
// come from inspector-built lists (u, q): u indexes row i, q is the position
// of L_jk.  Lane t gathers its list into a private LDS row M[t][u] = L_{j_t,k_u};
// the entries of row i are then resolved in ascending u: the lane owning u
// divides by its pivot L_jj, the value is broadcast inside the group, and
// every lane t > u subtracts M[t][u] * L_iu -- the same terms in the same
// ascending order as the recurrence above.
#include "dev_common.h"

namespace sf {
namespace {

using dev::after_wait;
using dev::group_sum;
using dev::ld_co;
using dev::st_co;
using dev::stores_complete;
using dev::wait_flag;

template <int G, bool FLAGS>
__device__ __forceinline__ void ic0_rows(const Ic0Args& a, int q0, int q1, int lane, double* lds_row) {
  constexpr int RPB = 64 / G;
  const int sub = lane & (G - 1);
  const int32_t par = a.ls.epoch & 1;
  for (int base = q0; base < q1; base += RPB) {
    const int q = base + lane / G;
    const bool act = q < q1;
    const int i = act ? a.order[q] : 0;
    const int r0 = act ? a.Lrp[i] : 0;
    const int rd = act ? a.Lrp[i + 1] - 1 : 0;  // diagonal position
    const int len = rd - r0;                     // off-diagonal entries (<= G)
    const bool mine = act && sub < len;
    const int p = r0 + sub;
    const int j = mine ? a.Lci[p] : 0;
    double l = 0.0;
    if (a.factor) {
      double acc = mine ? a.Aval[p] : 0.0;
      if constexpr (FLAGS) {
        if (mine) wait_flag(a.flags + j, a.ls);
        after_wait();
      }
      const double djj = mine ? ld_co(a.Lval + (a.Lrp[j + 1] - 1)) : 1.0;
      // private LDS row M[t][0..G): the factor entries L_{j_t, k_u}
      for (int u = 0; u < G; ++u) lds_row[u] = 0.0;
      if (mine) {
        const int e0 = a.pair_ptr[p], e1 = a.pair_ptr[p + 1];
        for (int e = e0; e < e1; ++e) lds_row[a.pair_u[e]] = ld_co(a.Lval + a.pair_q[e]);
      }
      // longest row of this batch bounds the sweep (wave-uniform)
      int maxlen = act ? len : 0;
      for (int off = 32; off >= 1; off >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, off, 64));
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (u >= maxlen) break;
        if (sub == u) l = acc / djj;  // entry u is final: every k < j_u was subtracted
        const double lu = __shfl(l, u, G);
        if (mine && sub > u) acc -= lds_row[u] * lu;
      }
      if (mine) st_co(a.Lval + p, l);
      const double sq = group_sum<G>(mine ? l * l : 0.0);
      const double piv = act ? a.Aval[rd] - sq : 1.0;
      const double lii = sqrt(piv);
      if (act && sub == 0) {
        if (!(piv > 0.0))
          __hip_atomic_fetch_min(a.ls.state + info_off(par), i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st_co(a.Lval + rd, lii);
      }
      if (a.solve) {
        double s = 0.0;
        if (mine) s = l * ld_co(a.X + j);
        s = group_sum<G>(s);
        if (act && sub == 0) st_co(a.X + i, (a.B[i] - s) / lii);
      }
    } else {
      // solve only, with a factor already in Lval
      if constexpr (FLAGS) {
        if (mine) wait_flag(a.flags + j, a.ls);
        after_wait();
      }
      double s = mine ? ld_co(a.Lval + p) * ld_co(a.X + j) : 0.0;
      s = group_sum<G>(s);
      if (act && sub == 0) st_co(a.X + i, (a.B[i] - s) / ld_co(a.Lval + rd));
    }
    if constexpr (FLAGS) {
      stores_complete();
      if (act && sub == 0) st_co(a.flags + i, a.ls.epoch);
    }
  }
}

__device__ __forceinline__ void write_info(const Ic0Args& a, int lane) {
  if (!a.d_info) return;
  if (dev::last_wave_done(a.ls, lane) && lane == 0) {
    const int32_t v = __hip_atomic_load(a.ls.state + info_off(a.ls.epoch & 1), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    *a.d_info = (v >= a.n) ? -1 : v;
  }
}

template <int G>
__global__ __launch_bounds__(kBlockThreads) void k_ic0_fused(Ic0Args a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  double* lds_row = lds + size_t(threadIdx.x) * G;
  dev::reset_next_launch(a.ls);
  for (;;) {
    const int t = dev::claim(a.ls, lane);
    if (t >= a.n_work) break;
    const int it = a.item_list ? a.item_list[t] : t;
    ic0_rows<G, true>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, lds_row);
  }
  write_info(a, lane);
}

template <int G>
__global__ __launch_bounds__(kBlockThreads) void k_ic0_levelset(Ic0Args a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  double* lds_row = lds + size_t(threadIdx.x) * G;
  dev::reset_next_launch(a.ls);
  const int wave = int(blockIdx.x) * (kBlockThreads / 64) + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * (kBlockThreads / 64);
  int32_t gen = 0;
  for (int lv = 0; lv < a.depth; ++lv) {
    for (int t = a.lvl_item_ptr[lv] + wave; t < a.lvl_item_ptr[lv + 1]; t += nwaves) {
      const int it = a.item_list[t];
      ic0_rows<G, false>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, lds_row);
    }
    if (lv + 1 < a.depth) dev::grid_barrier(a.ls, gen);
  }
  write_info(a, lane);
}

template <typename K>
int occ(K kernel, size_t lds) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(kernel),
                                                   kBlockThreads, lds) != hipSuccess)
    return 1;
  return b < 1 ? 1 : b;
}

}  // namespace

hipError_t launch_ic0_fused(const Ic0Args& a, int g, int grid, hipStream_t st) {
  const size_t lds = size_t(kBlockThreads) * g * sizeof(double);
#define SF_IC(G)                                                                    \
  if (g == G) {                                                                     \
    hipLaunchKernelGGL((k_ic0_fused<G>), dim3(grid), dim3(kBlockThreads), lds, st, a); \
    return hipGetLastError();                                                       \
  }
  SF_IC(4) SF_IC(8) SF_IC(16) SF_IC(32) SF_IC(64)
#undef SF_IC
  return hipErrorInvalidValue;
}

hipError_t launch_ic0_levelset(const Ic0Args& a, int g, int grid, hipStream_t st) {
  const size_t lds = size_t(kBlockThreads) * g * sizeof(double);
  void* args[] = {const_cast<Ic0Args*>(&a)};
#define SF_IL(G)                                                                               \
  if (g == G)                                                                                  \
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_ic0_levelset<G>), dim3(grid), \
                                      dim3(kBlockThreads), args, lds, st);
  SF_IL(4) SF_IL(8) SF_IL(16) SF_IL(32) SF_IL(64)
#undef SF_IL
  return hipErrorInvalidValue;
}

int occupancy_ic0(int g, int levelset) {
  const size_t lds = size_t(kBlockThreads) * g * sizeof(double);
  switch (g) {
    case 4: return levelset ? occ(k_ic0_levelset<4>, lds) : occ(k_ic0_fused<4>, lds);
    case 8: return levelset ? occ(k_ic0_levelset<8>, lds) : occ(k_ic0_fused<8>, lds);
    case 16: return levelset ? occ(k_ic0_levelset<16>, lds) : occ(k_ic0_fused<16>, lds);
    case 32: return levelset ? occ(k_ic0_levelset<32>, lds) : occ(k_ic0_fused<32>, lds);
    default: return levelset ? occ(k_ic0_levelset<64>, lds) : occ(k_ic0_fused<64>, lds);
  }
}

}  // namespace sf
