// Device probes: the machine constants that bound the executors, measured on
// the current device (sf_device_probe).
//   copy    stream copy of 1 GiB into 1 GiB: the practical HBM ceiling;
//   hop     one-way latency of a published value between two workgroups,
//           with the executors' protocol (the value itself is the readiness
//           flag: device-coherent store, device-coherent polling load), on
//           one XCD and across XCDs: the cost of one edge of a critical path;
//   gather  a dependence-free product sum over uniformly random columns of a
//           2^20-entry FP64 vector (50M gathers, coalesced column and value
//           streams): the rate of single-value gathers, which bounds any
//           schedule whose x reads have no locality.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "probe.h"

namespace sf {
namespace {

__device__ __forceinline__ unsigned xcc_id() {
  // hardware register XCC_ID (20), bits [3:0]
  return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));
}

__global__ void k_probe_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n4) {
  size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (; i < n4; i += stride) b[i] = a[i];
}

// Workgroups a and b exchange the values 1..iters through two slots on
// separate 256-byte lines; every other workgroup returns at once.  A poll
// that sees no new value within `limit` reads gives up and ends the loop,
// so the kernel always finishes.  out[0]: elapsed 100 MHz ticks on a,
// out[1]: 1 if a poll gave up, out[2], out[3]: XCC ids of a and b.
__global__ void k_probe_hop(double* slots, long long* out, int a, int b, int iters, int limit) {
  if (threadIdx.x != 0) return;
  const int me = blockIdx.x;
  if (me != a && me != b) return;
  double* ab = slots;
  double* ba = slots + 32;
  bool gave_up = false;
  const long long t0 = __builtin_amdgcn_s_memrealtime();
  for (int k = 1; k <= iters && !gave_up; ++k) {
    double* mine = me == a ? ab : ba;
    const double* theirs = me == a ? ba : ab;
    if (me == a) __hip_atomic_store(mine, double(k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int s = 0;
    while (__hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != double(k)) {
      if (++s > limit) {
        gave_up = true;
        break;
      }
    }
    if (me == b && !gave_up) __hip_atomic_store(mine, double(k), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  const long long t1 = __builtin_amdgcn_s_memrealtime();
  if (me == a) {
    out[0] = t1 - t0;
    out[2] = xcc_id();
  } else {
    out[3] = xcc_id();
  }
  if (gave_up) out[1] = 1;
}

// Column of entry k: a 64-bit multiply / xor-shift mix of k, modulo n.
__global__ void k_probe_gather_fill(int32_t* col, double* val, double* x, long long nnz, int32_t n) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < nnz; i += stride) {
    unsigned long long h = (unsigned long long)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    col[i] = int32_t(h % (unsigned long long)n);
    val[i] = 1.0 / double(1 + (i & 15));
    if (i < n) x[i] = double(i & 1023);
  }
}

// Each wavefront takes chunks of 64 U entries, entry u * 64 + lane of a
// chunk on each lane; the U column and value loads stream past the caches,
// then the U gathers are issued before any is used.
template <int U>
__global__ void k_probe_gather(const int32_t* __restrict__ col, const double* __restrict__ val, const double* x,
                               double* out, long long nnz) {
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const long long wave = tid >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  double acc = 0.0;
  for (long long chunk = wave * 64 * U; chunk < nnz; chunk += nwaves * 64 * U) {
    int32_t c[U];
    double v[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long e = chunk + u * 64 + lane;
      const bool in = e < nnz;
      c[u] = in ? __builtin_nontemporal_load(col + e) : -1;
      v[u] = in ? __builtin_nontemporal_load(val + e) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = c[u] < 0 ? 0.0 : x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u] * xv[u];
  }
  out[tid] = acc;
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

struct Buffers {
  void* p[4] = {nullptr, nullptr, nullptr, nullptr};
  ~Buffers() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
};

#define PROBE_HIP(x)                        \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

template <typename F>
hipError_t time_launches(F launch, int warm, int reps, hipStream_t st, double* ms) {
  Events ev;
  PROBE_HIP(hipEventCreate(&ev.e0));
  PROBE_HIP(hipEventCreate(&ev.e1));
  for (int w = 0; w < warm; ++w) launch();
  PROBE_HIP(hipGetLastError());
  PROBE_HIP(hipEventRecord(ev.e0, st));
  for (int r = 0; r < reps; ++r) launch();
  PROBE_HIP(hipGetLastError());
  PROBE_HIP(hipEventRecord(ev.e1, st));
  PROBE_HIP(hipEventSynchronize(ev.e1));
  float t = 0.f;
  PROBE_HIP(hipEventElapsedTime(&t, ev.e0, ev.e1));
  *ms = double(t) / reps;
  return hipSuccess;
}

}  // namespace

hipError_t probe_copy(int cus, hipStream_t st, double* gbps) {
  const size_t bytes = size_t(1) << 30;
  Buffers b;
  PROBE_HIP(hipMalloc(&b.p[0], bytes));
  PROBE_HIP(hipMalloc(&b.p[1], bytes));
  PROBE_HIP(hipMemsetAsync(b.p[0], 0, bytes, st));
  const size_t n4 = bytes / sizeof(float4);
  const float4* src = static_cast<const float4*>(b.p[0]);
  float4* dst = static_cast<float4*>(b.p[1]);
  double ms = 0.0;
  PROBE_HIP(time_launches([&] { hipLaunchKernelGGL(k_probe_copy, dim3(cus * 16), dim3(256), 0, st, src, dst, n4); },
                          3, 10, st, &ms));
  *gbps = 2.0 * double(bytes) / (ms * 1e-3) / 1e9;
  return hipSuccess;
}

hipError_t probe_hop(hipStream_t st, double* same_us, double* cross_us) {
  *same_us = *cross_us = -1.0;
  Buffers b;
  PROBE_HIP(hipMalloc(&b.p[0], 4096));
  PROBE_HIP(hipMalloc(&b.p[1], 64 * sizeof(long long)));
  double* slots = static_cast<double*>(b.p[0]);
  long long* out = static_cast<long long*>(b.p[1]);
  const int iters = 2000, limit = 1 << 20;
  // workgroups are dealt to the XCDs in turn, so 0 and 8 usually share one
  // and 0 and 1 usually do not; the XCC ids read back decide
  const int partner[2] = {8, 1};
  for (int k = 0; k < 2; ++k) {
    PROBE_HIP(hipMemsetAsync(slots, 0, 4096, st));
    PROBE_HIP(hipMemsetAsync(out, 0, 64 * sizeof(long long), st));
    hipLaunchKernelGGL(k_probe_hop, dim3(16), dim3(64), 0, st, slots, out, 0, partner[k], iters, limit);
    PROBE_HIP(hipGetLastError());
    long long h[4];
    PROBE_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, st));
    PROBE_HIP(hipStreamSynchronize(st));
    if (h[1] != 0) continue;  // a partner did not answer in time: no figure
    const double us = double(h[0]) * 0.01 / (2.0 * iters);  // 100 MHz ticks, two hops per exchange
    if (h[2] == h[3]) *same_us = us;
    else *cross_us = us;
  }
  return hipSuccess;
}

hipError_t probe_gather(int cus, hipStream_t st, double* per_s) {
  const int32_t n = 1 << 20;
  const long long nnz = 50000000;
  const int waves_per_cu = 8;
  const int grid = cus * waves_per_cu / 4;  // 256-thread workgroups
  Buffers b;
  PROBE_HIP(hipMalloc(&b.p[0], size_t(nnz) * sizeof(int32_t)));
  PROBE_HIP(hipMalloc(&b.p[1], size_t(nnz) * sizeof(double)));
  PROBE_HIP(hipMalloc(&b.p[2], size_t(n) * sizeof(double)));
  PROBE_HIP(hipMalloc(&b.p[3], size_t(grid) * 256 * sizeof(double)));
  int32_t* col = static_cast<int32_t*>(b.p[0]);
  double* val = static_cast<double*>(b.p[1]);
  double* x = static_cast<double*>(b.p[2]);
  double* out = static_cast<double*>(b.p[3]);
  hipLaunchKernelGGL(k_probe_gather_fill, dim3(cus * 8), dim3(256), 0, st, col, val, x, nnz, n);
  PROBE_HIP(hipGetLastError());
  double ms = 0.0;
  PROBE_HIP(time_launches(
      [&] { hipLaunchKernelGGL(k_probe_gather<8>, dim3(grid), dim3(256), 0, st, col, val, x, out, nnz); }, 3, 10,
      st, &ms));
  *per_s = double(nnz) / (ms * 1e-3);
  return hipSuccess;
}

}  // namespace sf
