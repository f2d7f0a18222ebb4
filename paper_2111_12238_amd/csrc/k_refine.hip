// Passes of the mixed-precision refinement (FP32 solves, FP64 residuals).
//
//   residual:  x_new = x + d (FP64), r = b - L64 x_new (FP64 values and
//              accumulation), r32 = (float) r; x_new is written to a second
//              buffer so rows never read a partly updated iterate.
//   final:     x_final = x + d, y = A64 x_final and r = b - L64 x_final in
//              FP64, plus max_i |r_i| and max_i |b_i| per column.
// Every vector is kept in the interleaved block layout of the multi-RHS
// solve (k_layout.hip), so one gather of a column index brings the KB values
// of a block's right-hand sides together and each row's reads and writes
// are contiguous.  KB lanes per row, one per right-hand side of the block,
// 64 / KB rows per wavefront; each lane runs its row's entries kR at a time
// (indices and values, then the iterate).  No dependences: every read is of
// finished data.
#include "dev_common.h"

namespace sf {
namespace {

constexpr int kR = 8;

template <int KB>
struct Layout {
  int32_t n;
  size_t boff;  // offset of (row 0, this lane's column) in the interleaved arrays
  __device__ __forceinline__ size_t at(int j) const { return boff + size_t(j) * KB; }
};

template <int KB>
__device__ __forceinline__ double xval(const ResArgs& a, const Layout<KB>& lay, int j) {
  const size_t k = lay.at(j);
  double v = a.xin ? a.xin[k] : 0.0;
  if (a.d) v += double(a.d[k]);
  return v;
}

// sum_p val[p] * (x + d)(col[p]) over p in [p0, p1), ascending
template <int KB>
__device__ __forceinline__ double row_dot(const ResArgs& a, const Layout<KB>& lay, const int32_t* __restrict__ col,
                                          const double* __restrict__ val, int p0, int p1) {
  double s = 0.0;
  for (int c0 = p0; c0 < p1; c0 += kR) {
    int j[kR];
    double v[kR], x[kR];
#pragma unroll
    for (int u = 0; u < kR; ++u) {
      const bool h = c0 + u < p1;
      j[u] = h ? col[c0 + u] : -1;
      v[u] = h ? val[c0 + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kR; ++u) x[u] = j[u] >= 0 ? xval<KB>(a, lay, j[u]) : 0.0;
#pragma unroll
    for (int u = 0; u < kR; ++u) s += v[u] * x[u];
  }
  return s;
}

// Maxima of |r| and |b| are kept as bit patterns (non-negative doubles order
// like their bit patterns): per block in LDS, then one device atomic per
// column and block (64 right-hand sides at most).
template <bool FINAL, int KB>
__global__ __launch_bounds__(kBlockThreads) void k_resid(ResArgs a) {
  constexpr int RPW = 64 / KB;
  __shared__ unsigned long long smax[FINAL ? 2 * 64 : 1];
  const int lane = threadIdx.x & 63;
  const int c = lane % KB;
  const int wave = int(blockIdx.x) * (kBlockThreads / 64) + int(threadIdx.x >> 6);
  const int nwaves = int(gridDim.x) * (kBlockThreads / 64);
  const int rows = FINAL ? max(a.n, a.m) : a.n;
  const int nblk = (a.nrhs + KB - 1) / KB;
  const int ngroups = (rows + RPW - 1) / RPW;
  if (FINAL) {
    for (int k = threadIdx.x; k < 2 * 64; k += kBlockThreads) smax[k] = 0ull;
    __syncthreads();
  }
  for (int u = wave; u < ngroups * nblk; u += nwaves) {
    const int blk = u % nblk;
    const int i = (u / nblk) * RPW + lane / KB;
    const int cc = blk * KB + c;
    const bool colok = cc < a.nrhs;
    Layout<KB> lay{a.n, size_t(blk) * size_t(a.n) * KB + c};
    if (i < a.n) {
      const double s = row_dot<KB>(a, lay, a.Lci, a.L64, a.Lrp[i], a.Lrp[i + 1]);
      const double b = a.B[lay.at(i)];  // zero in the padding columns of the last block
      const double r = b - s;
      const double xi = xval<KB>(a, lay, i);
      a.xout[lay.at(i)] = xi;
      if (FINAL) {
        if (colok) {
          atomicMax(&smax[2 * cc], (unsigned long long)__double_as_longlong(fabs(r)));
          atomicMax(&smax[2 * cc + 1], (unsigned long long)__double_as_longlong(fabs(b)));
        }
      } else {
        a.r32[lay.at(i)] = float(r);
      }
    }
    if (FINAL && a.Y && i < a.m) {
      const double y = row_dot<KB>(a, lay, a.Aci, a.A64, a.Arp[i], a.Arp[i + 1]);
      a.Y[size_t(blk) * size_t(a.m) * KB + size_t(i) * KB + c] = y;
    }
  }
  if (FINAL) {
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * a.nrhs; k += kBlockThreads)
      if (a.maxabs && smax[k] != 0ull)
        __hip_atomic_fetch_max(a.maxabs + k, smax[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ void k_convert(const double* src, float* dst, int32_t n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) dst[k] = float(src[k]);
}

__global__ void k_fill_u64(unsigned long long* p, int32_t count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) p[k] = 0ull;
}

template <bool FINAL>
hipError_t launch_resid(const ResArgs& a, hipStream_t st) {
  const int rows = FINAL ? (a.n > a.m ? a.n : a.m) : a.n;
  const int kb = a.kb;
  const size_t units = size_t((rows + 64 / kb - 1) / (64 / kb)) * size_t((a.nrhs + kb - 1) / kb);
  size_t g = (units + kBlockThreads / 64 - 1) / (kBlockThreads / 64);
  // the final pass issues one maxima atomic per column and block: cap its grid
  g = g < 1 ? 1 : (g > (FINAL ? 2048 : 8192) ? (FINAL ? 2048 : 8192) : g);
#define SF_RS(KB)                                                                         \
  if (kb == KB) {                                                                         \
    hipLaunchKernelGGL((k_resid<FINAL, KB>), dim3(unsigned(g)), dim3(kBlockThreads), 0, st, a); \
    return hipGetLastError();                                                             \
  }
  SF_RS(1) SF_RS(2) SF_RS(4) SF_RS(8) SF_RS(16) SF_RS(32) SF_RS(64)
#undef SF_RS
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_residual(const ResArgs& a, hipStream_t st) { return launch_resid<false>(a, st); }

hipError_t launch_final(const ResArgs& a, hipStream_t st) { return launch_resid<true>(a, st); }

hipError_t launch_convert_f64_f32(const double* src, float* dst, int32_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (n + 255) / 256;
  grid = grid > 8192 ? 8192 : grid;
  hipLaunchKernelGGL(k_convert, dim3(grid), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int32_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u64, dim3((count + 255) / 256), dim3(256), 0, st, p, count);
  return hipGetLastError();
}

}  // namespace sf
