// Fused SpILU0 -> SpTRSV executor (FP64) and its level-set baseline.
//
// Row i of the zero fill-in incomplete LU factors (Table 2, comb. 6) on
// the pattern P of A, by row-wise elimination restricted to P: for the
// stored columns k < i of row i in ascending order,
//     l_ik = (a_ik - sum_{m<k, m in P_i, (m,k) in P} l_im u_mk) / u_kk
// and for the stored j >= i
//     u_ij =  a_ij - sum_{m<i, m in P_i, (m,j) in P} l_im u_mj,
// each sum in ascending m; then, in the same work item (F = I: the solve of
// row i needs only factor rows it already reads), the unit-lower solve
//     y_i = x_i - sum_{k<i} l_ik y_k.
// L (unit diagonal implied) and U are returned in A's CSR positions.
//
// G lanes per row, lane t owns the t-th stored entry (diagonal and upper
// entries included; rows longer than G are rejected by the caller).  The
// intersections come from inspector-built lists (t << 16 | u, q): entry t
// of row i meets entry u (column k_u) where row k_u stores (k_u, j_t), at
// position q.  Lane t gathers them into a private LDS row M[t][u] = u_{k_u
// j_t}; the lower entries of the row are then resolved in ascending u: the
// lane owning u divides by its pivot u_{k_u k_u}, the value is broadcast in
// the group, every lane t > u with a pair at u subtracts M[t][u] * l_iu,
// and the row's first lane subtracts l_iu y_{k_u} from x_i -- every term of
// the recurrences above, rounded once, in their order, so FP64 results
// equal the sequential definition's bit for bit.
//
// Readiness (fused launch): the factor values and y are pre-filled with the
// pending pattern and every value is its own flag; a batch issues all its
// loads, then waits for the pending ones together (dev::wait_ptrs).  The
// level-set baseline factors with one grid barrier per level, then solves
// in a second level-set launch (factor = 0: L read, not computed).
#pragma clang fp contract(off)

#include "stream.h"

namespace sf {
namespace {

using dev::is_pending;
using dev::ld_co;
using dev::publishable;
using dev::st_co;

// Marker of an absent (t, u) pair in the LDS rows (a signalling NaN with a
// payload no stored factor value can carry: arithmetic returns NaNs quiet).
constexpr unsigned long long kAbsentBits = 0xFFF4000000000002ull;
constexpr double kAbsent = __builtin_bit_cast(double, kAbsentBits);
__device__ __forceinline__ bool is_absent(double v) {
  return __builtin_bit_cast(unsigned long long, v) == kAbsentBits;
}

constexpr int kPairRegs = 8;  // pairs gathered per lane and round

// LDS: lane t keeps M[t][u] for u < t only (a pair's lower entry precedes
// the entry it serves, entries being in column order); the G lanes of a
// row share a triangle of G (G - 1) / 2 doubles at group_lds.
template <int G>
constexpr int tri_size() { return G * (G - 1) / 2; }
__device__ __forceinline__ int tri_row(int t) { return t * (t - 1) / 2; }

template <int G, bool FUSED>
__device__ __forceinline__ void ilu_rows(const Ic0Args& a, int q0, int q1, int lane, double* group_lds) {
  constexpr int RPB = 64 / G;
  const int sub = lane & (G - 1);
  double* lds_row = group_lds + tri_row(sub);
  const int32_t par = a.ls.epoch & 1;
  for (int base = q0; base < q1; base += RPB) {
    const int q = base + lane / G;
    const bool act = q < q1;
    const int i = act ? a.order[q] : 0;
    const int r0 = act ? a.Lrp[i] : 0;
    const int r1 = act ? a.Lrp[i + 1] : 0;
    const int len = r1 - r0;  // stored entries of row i (<= G)
    const bool mine = act && sub < len;
    const int p = r0 + sub;
    const int j = mine ? a.Lci[p] : 0;
    const bool lower = mine && j < i;
    const int pjj = lower ? a.dpos[j] : 0;  // pivot u_jj
    const int nlow = act ? a.dpos[i] - r0 : 0;  // lower entries of row i come first
    const int e0 = act ? a.pair_ptr[r0] : 0, e1 = act ? a.pair_ptr[r1] : 0;
    double acc = (mine && a.factor) ? a.Aval[p] : 0.0;
    for (int u = 0; u < G; ++u)
      if (u < sub) lds_row[u] = kAbsent;
    __builtin_amdgcn_wave_barrier();
    int nround = a.factor ? (e1 - e0 + G * kPairRegs - 1) / (G * kPairRegs) : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) nround = max(nround, __shfl_xor(nround, off, 64));
    double djj = 1.0, yj = 0.0, lval = 0.0;
    for (int rnd = 0; rnd < (nround > 0 ? nround : 1); ++rnd) {
      constexpr int R = kPairRegs + 2;
      const double* ptr[R];
      double v[R];
      int tu[kPairRegs];
#pragma unroll
      for (int k = 0; k < kPairRegs; ++k) {
        const int e = e0 + rnd * G * kPairRegs + sub + G * k;
        const bool h = a.factor && e < e1;
        tu[k] = h ? a.pair_u[e] : -1;
        ptr[k] = h ? a.Lval + a.pair_q[e] : nullptr;
      }
      // factor: the pivot u_jj; solve only: the final l_ij itself
      ptr[kPairRegs] = (rnd == 0 && lower) ? a.Lval + (a.factor ? pjj : p) : nullptr;
      ptr[kPairRegs + 1] = (rnd == 0 && lower && a.solve) ? a.X + j : nullptr;
#pragma unroll
      for (int e = 0; e < R; ++e) v[e] = ptr[e] ? ld_co(ptr[e]) : 0.0;
      if constexpr (FUSED) dev::wait_ptrs<double, R, 64>(ptr, v, lane, a.ls);
#pragma unroll
      for (int k = 0; k < kPairRegs; ++k)
        if (tu[k] >= 0) group_lds[tri_row(tu[k] >> 16) + (tu[k] & 0xffff)] = v[k];
      if (rnd == 0 && lower) {
        if (a.factor) djj = v[kPairRegs];
        else lval = v[kPairRegs];
        if (a.solve) yj = v[kPairRegs + 1];
      }
    }
    __builtin_amdgcn_wave_barrier();
    int maxlow = act ? nlow : 0;  // the sweep covers the lower entries (wave-uniform bound)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) maxlow = max(maxlow, __shfl_xor(maxlow, off, 64));
    double s = (act && a.solve) ? a.B[i] : 0.0;  // right-hand side, on the row's first lane
#pragma unroll
    for (int u = 0; u < G; ++u) {
      if (u >= maxlow) break;
      double pr = 0.0;
      if (sub == u && lower) {  // entry u is final: every m < k_u has been subtracted
        if (a.factor) lval = acc / djj;
        pr = lval * yj;
      }
      const double lu = __shfl(lval, u, G);
      const double pu = __shfl(pr, u, G);
      if (a.factor && mine && sub > u) {
        const double m = lds_row[u];
        if (!is_absent(m)) acc = acc - m * lu;
      }
      if (act && sub == 0 && u < nlow) s = s - pu;
    }
    if (a.factor && mine) {
      st_co(a.Lval + p, publishable(lower ? lval : acc));
      if (j == i && !(acc != 0.0))
        __hip_atomic_fetch_min(a.ls.state + info_off(par), i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (act && sub == 0 && a.solve) st_co(a.X + i, publishable(s));
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
__global__ __launch_bounds__(kBlockThreads) void k_ilu0_fused(Ic0Args a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  double* group_lds = lds + size_t(threadIdx.x / G) * tri_size<G>();
  dev::reset_next_launch(a.ls);
  int t = dev::claim(a.ls, lane);
  while (t < a.n_work) {
    const int tn = dev::claim(a.ls, lane);  // prefetched (see k_ts_fused)
    const int it = a.item_list ? a.item_list[t] : t;
    ilu_rows<G, true>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, group_lds);
    t = tn;
  }
  write_info(a, lane);
}

template <int G>
__global__ __launch_bounds__(kBlockThreads) void k_ilu0_levelset(Ic0Args a) {
  extern __shared__ double lds[];
  const int lane = threadIdx.x & 63;
  double* group_lds = lds + size_t(threadIdx.x / G) * tri_size<G>();
  dev::reset_next_launch(a.ls);
  const int wave = int(blockIdx.x) * (kBlockThreads / 64) + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * (kBlockThreads / 64);
  int32_t gen = 0;
  for (int lv = 0; lv < a.depth; ++lv) {
    for (int t = a.lvl_item_ptr[lv] + wave; t < a.lvl_item_ptr[lv + 1]; t += nwaves) {
      const int it = a.item_list[t];
      ilu_rows<G, false>(a, a.item_ptr[it], a.item_ptr[it + 1], lane, group_lds);
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

hipError_t launch_ilu0_fused(const Ic0Args& a, int g, int grid, hipStream_t st) {
  if (!a.dpos || !a.order || !a.item_ptr || !a.pair_ptr) return hipErrorInvalidValue;
  const size_t lds = size_t(kBlockThreads / g) * size_t(g * (g - 1) / 2) * sizeof(double);
#define SF_IL(G)                                                                     \
  if (g == G) {                                                                      \
    hipLaunchKernelGGL((k_ilu0_fused<G>), dim3(grid), dim3(kBlockThreads), lds, st, a); \
    return hipGetLastError();                                                        \
  }
  SF_IL(4) SF_IL(8) SF_IL(16) SF_IL(32) SF_IL(64)
#undef SF_IL
  return hipErrorInvalidValue;
}

hipError_t launch_ilu0_levelset(const Ic0Args& a, int g, int grid, hipStream_t st) {
  if (!a.dpos || !a.order || !a.item_ptr || !a.pair_ptr || !a.item_list || !a.lvl_item_ptr)
    return hipErrorInvalidValue;
  const size_t lds = size_t(kBlockThreads / g) * size_t(g * (g - 1) / 2) * sizeof(double);
  void* args[] = {const_cast<Ic0Args*>(&a)};
#define SF_IL(G)                                                                                \
  if (g == G)                                                                                   \
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_ilu0_levelset<G>), dim3(grid), \
                                      dim3(kBlockThreads), args, lds, st);
  SF_IL(4) SF_IL(8) SF_IL(16) SF_IL(32) SF_IL(64)
#undef SF_IL
  return hipErrorInvalidValue;
}

int occupancy_ilu0(int g, int levelset) {
  const size_t lds = size_t(kBlockThreads / g) * size_t(g * (g - 1) / 2) * sizeof(double);
  switch (g) {
    case 4: return levelset ? occ(k_ilu0_levelset<4>, lds) : occ(k_ilu0_fused<4>, lds);
    case 8: return levelset ? occ(k_ilu0_levelset<8>, lds) : occ(k_ilu0_fused<8>, lds);
    case 16: return levelset ? occ(k_ilu0_levelset<16>, lds) : occ(k_ilu0_fused<16>, lds);
    case 32: return levelset ? occ(k_ilu0_levelset<32>, lds) : occ(k_ilu0_fused<32>, lds);
    default: return levelset ? occ(k_ilu0_levelset<64>, lds) : occ(k_ilu0_fused<64>, lds);
  }
}

}  // namespace sf
