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

// Maxima of |r| and |b| are kept as bit patterns: non-negative doubles
// order like their bit patterns.

// The final pass keeps the per-column maxima of a block in LDS and issues one
// device atomic per column and block at the end (64 right-hand sides max).
template <bool FINAL>
__global__ __launch_bounds__(kBlockThreads) void k_resid(ResArgs a) {
  constexpr int RPB = 64 / kG;
  __shared__ unsigned long long smax[FINAL ? 2 * 64 : 1];
  const int lane = threadIdx.x & 63;
  const int sub = lane & (kG - 1);
  const int wave = int(blockIdx.x) * (kBlockThreads / 64) + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * (kBlockThreads / 64);
  const int rows = FINAL ? max(a.n, a.m) : a.n;
  if (FINAL) {
    for (int k = threadIdx.x; k < 2 * 64; k += kBlockThreads) smax[k] = 0ull;
    __syncthreads();
  }
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
        if (i < a.n && sub == 0) {
          atomicMax(&smax[2 * c], (unsigned long long)__double_as_longlong(fabs(rmax)));
          atomicMax(&smax[2 * c + 1], (unsigned long long)__double_as_longlong(fabs(bmax)));
        }
      }
    }
  }
  if (FINAL) {
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * a.nrhs; k += kBlockThreads)
      if (a.maxabs && smax[k] != 0ull)
        __hip_atomic_fetch_max(a.maxabs + k, smax[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
  int grid = grid_for(a.n > a.m ? a.n : a.m);
  grid = grid > 2048 ? 2048 : grid;  // bounds the number of per-block maxima atomics
  hipLaunchKernelGGL((k_resid<true>), dim3(grid), dim3(kBlockThreads), 0, st, a);
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
