// Microbenchmarks behind two design choices of the executors (the machine
// constants that bound them -- copy ceiling, hop latency, gather rate -- are
// measured by the library itself, sf_device_probe):
//   pingpong  readiness-flag hop latency between two workgroups, for two
//             publication protocols (data + fence + flag, and
//             device-coherent data + flag), on the same XCD and across XCDs;
//   ticket    throughput of device-scope atomic work claiming on one
//             counter versus one counter per XCD.
// Output: one JSON object per line on stdout.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#define CK(x)                                                                   \
  do {                                                                          \
    hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                     \
      fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, \
              __LINE__);                                                        \
      exit(1);                                                                  \
    }                                                                           \
  } while (0)

__device__ __forceinline__ unsigned xcc_id() {
  // HW_REG_XCC_ID (hardware register 20), bits [3:0]
  return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11));
}

// Protocol 0: plain data store, agent release fence, relaxed flag store;
//             relaxed flag poll, agent acquire fence, plain data load.
// Protocol 1: device-coherent (agent-scope atomic) data store, wait for the
//             store to complete, device-coherent flag store; relaxed poll,
//             device-coherent data load (no cache-wide fences).
template <int PROTO>
__device__ __forceinline__ void publish(double* data, int* flag, double v, int k) {
  if (PROTO == 0) {
    *data = v;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flag, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    __hip_atomic_store(data, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __asm__ __volatile__("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(flag, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int PROTO>
__device__ __forceinline__ double consume(const double* data, const int* flag, int k,
                                          long long* spins, int limit, bool* gave_up) {
  int s = 0;
  while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != k) {
    if (++s > limit) {
      *gave_up = true;
      break;
    }
  }
  *spins += s;
  if (PROTO == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *(volatile const double*)data;
  } else {
    __asm__ __volatile__("" ::: "memory");
    return __hip_atomic_load(data, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Blocks a and b ping-pong `iters` times; every other block exits at once.
// out[0] = elapsed ticks of the 100 MHz real-time counter on block a,
// out[1] = mismatching data values seen, out[2..3] = XCC ids of a and b,
// out[4] = total spins, out[5] = 1 if a poll hit the spin limit.
template <int PROTO>
__global__ void pingpong(int* flags, double* data, long long* out, int a, int b, int iters,
                         int limit) {
  if (threadIdx.x != 0) return;
  int me = blockIdx.x;
  if (me != a && me != b) return;
  long long spins = 0, bad = 0;
  bool gave_up = false;
  int* f_ab = flags;         // a -> b
  int* f_ba = flags + 64;    // b -> a (own 256-byte line)
  double* d_ab = data;
  double* d_ba = data + 32;
  long long t0 = __builtin_amdgcn_s_memrealtime();
  for (int k = 1; k <= iters; ++k) {
    if (me == a) {
      publish<PROTO>(d_ab, f_ab, (double)k, k);
      double v = consume<PROTO>(d_ba, f_ba, k, &spins, limit, &gave_up);
      if (v != (double)k) ++bad;
    } else {
      double v = consume<PROTO>(d_ab, f_ab, k, &spins, limit, &gave_up);
      if (v != (double)k) ++bad;
      publish<PROTO>(d_ba, f_ba, (double)k, k);
    }
    if (gave_up) break;  // the partner is not answering: stop, never wait again
  }
  long long t1 = __builtin_amdgcn_s_memrealtime();
  if (me == a) {
    out[0] = t1 - t0;
    out[1] = bad;
    out[2] = xcc_id();
    out[4] = spins;
  } else {
    out[3] = xcc_id();
    out[6] = bad;
  }
  if (gave_up) out[5] = 1;
}

// Lane 0 of every wave claims `per_wave` tickets from counter[sel(block)].
__global__ void tickets(int* counters, int per_wave, int mode) {
  if ((threadIdx.x & 63) != 0) return;
  int c = 0;
  if (mode == 1) c = (blockIdx.x & 7) * 64;
  if (mode == 2) c = (int)xcc_id() * 64;
  int acc = 0;
  for (int k = 0; k < per_wave; ++k)
    acc += __hip_atomic_fetch_add(counters + c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (acc == -1) counters[1] = acc;  // keep the result live
}

int main(int argc, char** argv) {
  const char* what = argc > 1 ? argv[1] : "all";
  hipDeviceProp_t prop;
  CK(hipGetDeviceProperties(&prop, 0));
  printf("{\"device\": \"%s\", \"gcn\": \"%s\", \"cus\": %d, \"l2_bytes\": %d, \"clock_khz\": %d, "
         "\"mem_clock_khz\": %d, \"bus_width\": %d}\n",
         prop.name, prop.gcnArchName, prop.multiProcessorCount, prop.l2CacheSize, prop.clockRate,
         prop.memoryClockRate, prop.memoryBusWidth);
  fflush(stdout);
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));

  if (!strcmp(what, "all") || !strcmp(what, "pingpong")) {
    int* flags;
    double* data;
    long long* out;
    CK(hipMalloc(&flags, 4096));
    CK(hipMalloc(&data, 4096));
    CK(hipMalloc(&out, 64 * sizeof(long long)));
    const int iters = 2000, limit = 1 << 20;
    int pairs[2][2] = {{0, 8}, {0, 1}};
    for (int proto = 0; proto < 2; ++proto)
      for (int pi = 0; pi < 2; ++pi) {
        CK(hipMemset(flags, 0, 4096));
        CK(hipMemset(data, 0, 4096));
        CK(hipMemset(out, 0, 64 * sizeof(long long)));
        int a = pairs[pi][0], b = pairs[pi][1];
        auto t0 = std::chrono::steady_clock::now();
        if (proto == 0)
          pingpong<0><<<16, 64>>>(flags, data, out, a, b, iters, limit);
        else
          pingpong<1><<<16, 64>>>(flags, data, out, a, b, iters, limit);
        CK(hipDeviceSynchronize());
        auto t1 = std::chrono::steady_clock::now();
        long long h[8];
        CK(hipMemcpy(h, out, sizeof(h), hipMemcpyDeviceToHost));
        double us_rt = h[0] * 0.01 / iters;  // 100 MHz ticks -> us per round trip
        printf("{\"bench\": \"pingpong\", \"proto\": %d, \"blocks\": [%d, %d], \"xcc\": [%lld, %lld], "
               "\"hop_us\": %.3f, \"mismatch\": %lld, \"spin_limit_hit\": %lld, \"wall_ms\": %.2f}\n",
               proto, a, b, h[2], h[3], us_rt / 2, h[1] + h[6], h[5],
               std::chrono::duration<double, std::milli>(t1 - t0).count());
        fflush(stdout);
      }
    CK(hipFree(flags));
    CK(hipFree(data));
    CK(hipFree(out));
  }

  if (!strcmp(what, "all") || !strcmp(what, "ticket")) {
    int* counters;
    CK(hipMalloc(&counters, 64 * 64 * sizeof(int)));
    int grid = prop.multiProcessorCount * 4, per_wave = 64;
    for (int mode = 0; mode < 3; ++mode) {
      CK(hipMemset(counters, 0, 64 * 64 * sizeof(int)));
      tickets<<<grid, 256>>>(counters, per_wave, mode);
      CK(hipDeviceSynchronize());
      CK(hipEventRecord(e0));
      tickets<<<grid, 256>>>(counters, per_wave, mode);
      CK(hipEventRecord(e1));
      CK(hipEventSynchronize(e1));
      float ms;
      CK(hipEventElapsedTime(&ms, e0, e1));
      double total = (double)grid * 4 * per_wave;
      printf("{\"bench\": \"ticket\", \"mode\": %d, \"atomics\": %.0f, \"ms\": %.4f, \"ns_per_atomic\": %.3f}\n",
             mode, total, ms, ms * 1e6 / total);
      fflush(stdout);
    }
    CK(hipFree(counters));
  }

  return 0;
}
