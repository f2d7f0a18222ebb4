// Passes of the mixed-precision refinement (FP32 solves, FP64 residuals).
//
//   residual:  x_new = x + d (FP64), r = b - L64 x_new (FP64 values and
//              accumulation), r32 = (float) r; x_new is written to a second
//              buffer so rows never read a partly updated iterate.
//   final:     x_final = x + d, y = A64 x_final and r = b - L64 x_final in
//              FP64, plus max_i |r_i| and max_i |b_i| per column.
// Eight lanes per row (a whole 8-lane group always shares one row, so the
// group sums stay inside one branch); no dependences: all reads are of
// finished data.
#include "dev_common.h"

namespace sf {
namespace {

constexpr int kG = 8;
using dev::group_sum;

__device__ __forceinline__ double xval(const ResArgs& a, size_t k) {
  double v = a.xin ? a.xin[k] : 0.0;
  if (a.d) v += double(a.d[k]);
  return v;
}

// Non-negative doubles order like their bit patterns.
__device__ __forceinline__ void atomic_max_abs(unsigned long long* p, double v) {
  __hip_atomic_fetch_max(p, (unsigned long long)__double_as_longlong(fabs(v)), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

template <bool FINAL>
__global__ __launch_bounds__(kBlockThreads) void k_resid(ResArgs a) {
  constexpr int RPB = 64 / kG;
  const int lane = threadIdx.x & 63;
  const int sub = lane & (kG - 1);
  const int wave = int(blockIdx.x) * (kBlockThreads / 64) + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * (kBlockThreads / 64);
  const int rows = FINAL ? max(a.n, a.m) : a.n;
  for (int base = wave * RPB; base < rows; base += nwaves * RPB) {
    const int i = base + lane / kG;
    for (int c = 0; c < a.nrhs; ++c) {
      const size_t off = size_t(c) * size_t(a.n);
      double rmax = 0.0, bmax = 0.0;
      if (i < a.n) {
        double s = 0.0;
        for (int p = a.Lrp[i] + sub; p < a.Lrp[i + 1]; p += kG) s += a.L64[p] * xval(a, off + a.Lci[p]);
        s = group_sum<kG>(s);
        const double b = a.B[size_t(i) + size_t(c) * a.ldb];
        const double r = b - s;
        if (sub == 0) {
          a.xout[size_t(i) + size_t(c) * a.ldxo] = xval(a, off + i);
          if (a.r32) a.r32[off + i] = float(r);
        }
        rmax = r;
        bmax = b;
      }
      if (FINAL) {
        double y = 0.0;
        if (i < a.m)
          for (int p = a.Arp[i] + sub; p < a.Arp[i + 1]; p += kG) y += a.A64[p] * xval(a, off + a.Aci[p]);
        y = group_sum<kG>(y);
        if (i < a.m && sub == 0) a.Y[size_t(i) + size_t(c) * a.ldy] = y;
        if (i < a.n && sub == 0 && a.maxabs) {
          atomic_max_abs(a.maxabs + 2 * c, rmax);
          atomic_max_abs(a.maxabs + 2 * c + 1, bmax);
        }
      }
    }
  }
}

__global__ void k_convert(const double* src, int32_t lds, float* dst, int32_t n, int32_t nrhs) {
  const size_t total = size_t(n) * size_t(nrhs);
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < total;
       k += size_t(gridDim.x) * blockDim.x) {
    const size_t c = k / size_t(n), i = k - c * size_t(n);
    dst[k] = float(src[i + c * size_t(lds)]);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int32_t count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) p[k] = 0ull;
}

int grid_for(int rows) {
  const int per_block = (kBlockThreads / 64) * (64 / kG);
  int g = (rows + per_block - 1) / per_block;
  return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

}  // namespace

hipError_t launch_residual(const ResArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_resid<false>), dim3(grid_for(a.n)), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_final(const ResArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_resid<true>), dim3(grid_for(a.n > a.m ? a.n : a.m)), dim3(kBlockThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* src, int32_t lds, float* dst, int32_t n, int32_t nrhs,
                                  hipStream_t st) {
  const size_t total = size_t(n) * size_t(nrhs);
  int grid = int((total + 255) / 256);
  grid = grid < 1 ? 1 : (grid > 8192 ? 8192 : grid);
  hipLaunchKernelGGL(k_convert, dim3(grid), dim3(256), 0, st, src, lds, dst, n, nrhs);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int32_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

}  // namespace sf
