// Conversions between the caller's column-major right-hand-side blocks and
// the interleaved block layout the multi-RHS executors work in.
//
// Interleaved layout of `rows` x `ncols` values in blocks of KB columns:
// element (i, c), c = blk * KB + cb, sits at [(blk * rows + i) * KB + cb];
// columns past ncols (the tail of the last block) are zero.  One row of a
// block is then KB contiguous values, so a gather of x_j brings all of a
// block's right-hand sides in one access, and a row's reads and writes are
// coalesced whatever the order in which the executor visits rows.
//
// Both directions stage a tile of TR rows x KB columns in LDS: the
// column-major side is read or written along the rows (coalesced per
// column), the interleaved side along the tile's contiguous span.
#include "dev_common.h"

namespace sf {
namespace {

constexpr int kThreads = 256;

template <int KB>
struct Tile {
  static constexpr int rows = (2048 / KB) > 64 ? (2048 / KB) : 64;  // TR
  static constexpr int ld = KB + 1;                                  // LDS row pitch (bank spread)
};

// src column-major (ld lds, ncols columns) -> dst interleaved (converted to
// Tout); pend, when given, is filled with the pending pattern at the same
// positions (the multi-RHS solution buffer, which doubles as its flags).
template <typename Tin, typename Tout, int KB>
__global__ __launch_bounds__(kThreads) void k_pack(const Tin* __restrict__ src, int32_t lds, int32_t rows,
                                                   int32_t ncols, Tout* __restrict__ dst, Tout* __restrict__ pend) {
  using TL = Tile<KB>;
  __shared__ Tin t[TL::rows * TL::ld];
  const int nblk = (ncols + KB - 1) / KB;
  const int tiles_per_blk = (rows + TL::rows - 1) / TL::rows;
  const Tout pv = __builtin_bit_cast(Tout, dev::Pending<Tout>::bits);
  for (int tile = blockIdx.x; tile < nblk * tiles_per_blk; tile += gridDim.x) {
    const int blk = tile / tiles_per_blk;
    const int r0 = (tile - blk * tiles_per_blk) * TL::rows;
    for (int e = threadIdx.x; e < TL::rows * KB; e += kThreads) {
      const int r = e % TL::rows, cb = e / TL::rows;
      const int i = r0 + r, c = blk * KB + cb;
      t[r * TL::ld + cb] = (i < rows && c < ncols) ? src[size_t(i) + size_t(c) * size_t(lds)] : Tin(0);
    }
    __syncthreads();
    const size_t base = (size_t(blk) * size_t(rows) + size_t(r0)) * KB;
    for (int e = threadIdx.x; e < TL::rows * KB; e += kThreads) {
      const int r = e / KB, cb = e - r * KB;
      if (r0 + r < rows) {
        dst[base + e] = Tout(t[r * TL::ld + cb]);
        if (pend) pend[base + e] = pv;
      }
    }
    __syncthreads();
  }
}

// src interleaved -> dst column-major (ld ldd), the first ncols columns.
template <typename T, int KB>
__global__ __launch_bounds__(kThreads) void k_unpack(const T* __restrict__ src, int32_t rows, int32_t ncols,
                                                     T* __restrict__ dst, int32_t ldd) {
  using TL = Tile<KB>;
  __shared__ T t[TL::rows * TL::ld];
  const int nblk = (ncols + KB - 1) / KB;
  const int tiles_per_blk = (rows + TL::rows - 1) / TL::rows;
  for (int tile = blockIdx.x; tile < nblk * tiles_per_blk; tile += gridDim.x) {
    const int blk = tile / tiles_per_blk;
    const int r0 = (tile - blk * tiles_per_blk) * TL::rows;
    const size_t base = (size_t(blk) * size_t(rows) + size_t(r0)) * KB;
    for (int e = threadIdx.x; e < TL::rows * KB; e += kThreads) {
      const int r = e / KB, cb = e - r * KB;
      if (r0 + r < rows) t[r * TL::ld + cb] = src[base + e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TL::rows * KB; e += kThreads) {
      const int r = e % TL::rows, cb = e / TL::rows;
      const int i = r0 + r, c = blk * KB + cb;
      if (i < rows && c < ncols) dst[size_t(i) + size_t(c) * size_t(ldd)] = t[r * TL::ld + cb];
    }
    __syncthreads();
  }
}

int grid_for(int rows, int ncols, int kb) {
  const int tr = (2048 / kb) > 64 ? (2048 / kb) : 64;
  const long tiles = long((ncols + kb - 1) / kb) * long((rows + tr - 1) / tr);
  return int(tiles < 1 ? 1 : (tiles > 4096 ? 4096 : tiles));
}

template <typename Tin, typename Tout>
hipError_t pack_t(const void* src, int32_t lds, int32_t rows, int32_t ncols, void* dst, void* pend, int kb,
                  hipStream_t st) {
  const int grid = grid_for(rows, ncols, kb);
  const Tin* s = static_cast<const Tin*>(src);
  Tout* d = static_cast<Tout*>(dst);
  Tout* p = static_cast<Tout*>(pend);
#define SF_PK(KB)                                                                                   \
  if (kb == KB) {                                                                                   \
    hipLaunchKernelGGL((k_pack<Tin, Tout, KB>), dim3(grid), dim3(kThreads), 0, st, s, lds, rows, ncols, d, p); \
    return hipGetLastError();                                                                       \
  }
  SF_PK(2) SF_PK(4) SF_PK(8) SF_PK(16) SF_PK(32) SF_PK(64)
#undef SF_PK
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t unpack_t(const void* src, int32_t rows, int32_t ncols, void* dst, int32_t ldd, int kb, hipStream_t st) {
  const int grid = grid_for(rows, ncols, kb);
  const T* s = static_cast<const T*>(src);
  T* d = static_cast<T*>(dst);
#define SF_UP(KB)                                                                                \
  if (kb == KB) {                                                                                \
    hipLaunchKernelGGL((k_unpack<T, KB>), dim3(grid), dim3(kThreads), 0, st, s, rows, ncols, d, ldd); \
    return hipGetLastError();                                                                    \
  }
  SF_UP(2) SF_UP(4) SF_UP(8) SF_UP(16) SF_UP(32) SF_UP(64)
#undef SF_UP
  return hipErrorInvalidValue;
}

// Zero `ncols` columns of `rows` entries, column c at p + c * ld (a kernel,
// not a memset, so that the call can sit in a captured graph).
template <typename T>
__global__ void k_zero_cols(T* p, int32_t rows, int32_t ld, int32_t ncols) {
  const size_t count = size_t(rows) * size_t(ncols);
  for (size_t k = blockIdx.x * size_t(blockDim.x) + threadIdx.x; k < count; k += size_t(gridDim.x) * blockDim.x) {
    const size_t c = k / size_t(rows), i = k - c * size_t(rows);
    p[i + c * size_t(ld)] = T(0);
  }
}

}  // namespace

hipError_t launch_zero_cols(void* p, int32_t rows, int32_t ld, int32_t ncols, int dtype, hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (!p || ld < rows) return hipErrorInvalidValue;
  const size_t g = (size_t(rows) * size_t(ncols) + kThreads - 1) / kThreads;
  const int grid = int(g > 16384 ? 16384 : g);
  if (dtype == 0)
    hipLaunchKernelGGL(k_zero_cols<double>, dim3(grid), dim3(kThreads), 0, st, static_cast<double*>(p), rows, ld, ncols);
  else
    hipLaunchKernelGGL(k_zero_cols<float>, dim3(grid), dim3(kThreads), 0, st, static_cast<float*>(p), rows, ld, ncols);
  return hipGetLastError();
}

hipError_t launch_pack(const void* src, int src_dtype, int32_t lds, int32_t rows, int32_t ncols, void* dst,
                       int dst_dtype, void* pend, int kb, hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (!src || !dst || lds < rows) return hipErrorInvalidValue;
  if (src_dtype == 0 && dst_dtype == 0) return pack_t<double, double>(src, lds, rows, ncols, dst, pend, kb, st);
  if (src_dtype == 1 && dst_dtype == 1) return pack_t<float, float>(src, lds, rows, ncols, dst, pend, kb, st);
  if (src_dtype == 0 && dst_dtype == 1) return pack_t<double, float>(src, lds, rows, ncols, dst, pend, kb, st);
  return hipErrorInvalidValue;
}

hipError_t launch_unpack(const void* src, int dtype, int32_t rows, int32_t ncols, void* dst, int32_t ldd, int kb,
                         hipStream_t st) {
  if (rows <= 0 || ncols <= 0) return hipSuccess;
  if (!src || !dst || ldd < rows) return hipErrorInvalidValue;
  return dtype == 0 ? unpack_t<double>(src, rows, ncols, dst, ldd, kb, st)
                    : unpack_t<float>(src, rows, ncols, dst, ldd, kb, st);
}

}  // namespace sf
