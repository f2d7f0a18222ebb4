// Backward executor: the adjoint of y = A L^{-1} b in one persistent launch.
//
// With g = dloss/dy, the gradients are lambda = L^{-T} (A^T g), grad_b =
// lambda and grad_L = -(lambda x^T) on the pattern of L.  The transposed
// solve runs over its own schedule (reversed wavefronts of L^T).  Row i of
// the upper solve computes c_i = (A^T g)_i from row i of A^T on the spot
// (it depends on nothing: the paper's SpMV -> SpTRSV combination with the
// product interleaved into the solve), waits on the flags of the lambda_j,
// j > i, it reads, stores
//     lambda_i = (c_i - sum_{j>i} L_ji lambda_j) / L_ii,
// writes grad_L for every stored L_ik of row i of L (-lambda_i x_k, x is
// final input data), then publishes its flag.  Values of L^T and A^T are
// read through the inspector's transpose maps; grad_L is written in the
// CSR order of L.
#include "dev_common.h"

namespace sf {
namespace {

using dev::after_wait;
using dev::group_sum;
using dev::ld_co;
using dev::st_co;
using dev::stores_complete;
using dev::wait_flag;

template <typename T, int G>
__global__ __launch_bounds__(kBlockThreads) void k_bwd(BwdArgs a) {
  constexpr int RPB = 64 / G;
  const int lane = threadIdx.x & 63;
  const int sub = lane & (G - 1);
  const T* __restrict__ Lv = static_cast<const T*>(a.Lv);
  const T* __restrict__ Av = static_cast<const T*>(a.Av);
  const T* __restrict__ X = static_cast<const T*>(a.X);
  const T* __restrict__ Gv = static_cast<const T*>(a.G);
  T* lam = static_cast<T*>(a.lam);
  T* __restrict__ gL = static_cast<T*>(a.gradL);
  dev::reset_next_launch(a.ls);
  for (;;) {
    const int t = dev::claim(a.ls, lane);
    if (t >= a.n_work) break;
    const int q0 = a.item_ptr[t], q1 = a.item_ptr[t + 1];
    for (int base = q0; base < q1; base += RPB) {
      const int q = base + lane / G;
      const bool act = q < q1;
      const int i = act ? a.order[q] : 0;
      // c_i = sum_r A_ri g_r over row i of A^T
      T c = T(0);
      if (act)
        for (int e = a.ATrp[i] + sub; e < a.ATrp[i + 1]; e += G) c += Av[a.ATmap[e]] * Gv[a.ATci[e]];
      // row i of L^T: the diagonal first, then L_ji for j > i
      const int e0 = act ? a.LTrp[i] : 0;
      const int e1 = act ? a.LTrp[i + 1] : 0;
      T s = T(0);
      for (int eb = e0 + 1; eb < e1; eb += G) {
        const int e = eb + sub;
        const bool have = e < e1;
        const int j = have ? a.LTci[e] : 0;
        const T v = have ? Lv[a.LTmap[e]] : T(0);
        if (have) wait_flag(a.flags + j, a.ls);
        after_wait();
        if (have) s += v * ld_co(lam + j);
      }
      c = group_sum<G>(c);
      s = group_sum<G>(s);
      const T lii = act ? Lv[a.LTmap[e0]] : T(1);
      const T li = (c - s) / lii;  // the same value on every lane of the group
      if (act && sub == 0) st_co(lam + i, li);
      if (act)
        for (int p = a.Lrp[i] + sub; p < a.Lrp[i + 1]; p += G)
          __builtin_nontemporal_store(-li * X[a.Lci[p]], gL + p);
      stores_complete();
      if (act && sub == 0) st_co(a.flags + i, a.ls.epoch);
    }
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

template <typename T>
hipError_t bwd_dispatch(const BwdArgs& a, int g, int grid, hipStream_t st) {
#define SF_BW(G)                                                                   \
  if (g == G) {                                                                    \
    hipLaunchKernelGGL((k_bwd<T, G>), dim3(grid), dim3(kBlockThreads), 0, st, a); \
    return hipGetLastError();                                                      \
  }
  SF_BW(2) SF_BW(4) SF_BW(8) SF_BW(16) SF_BW(32)
#undef SF_BW
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_bwd(const BwdArgs& a, int dtype, int g, int grid, hipStream_t st) {
  return dtype == 0 ? bwd_dispatch<double>(a, g, grid, st) : bwd_dispatch<float>(a, g, grid, st);
}

int occupancy_bwd(int dtype, int g) {
  (void)g;
  return dtype == 0 ? occ(k_bwd<double, 8>) : occ(k_bwd<float, 8>);
}

}  // namespace sf
