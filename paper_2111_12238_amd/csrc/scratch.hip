// Fixed device scratch of the allocation-free entry point
// (sf_backward_noalloc): callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops) get the recomputed solution
// x of the adjoint from this array instead of a workspace argument.
//
// The array lives in the library's code object, so each GPU the library
// runs on holds its own copy (kScratchBytes) from module load until the
// process ends.  In host code the array's name is not a device address:
// the address is looked up once per device with hipGetSymbolAddress, with
// that device current, and kept per device; only that address is ever
// handed to kernels.  Every call on one GPU shares its array, so calls that
// overlap on one GPU race (they must be ordered on one stream or otherwise
// serialised).
#include <hip/hip_runtime.h>

#include <mutex>

#include "kargs.h"

namespace sf {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 8M FP64 (16M FP32) values
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t scratch_bytes() { return kScratchBytes; }

hipError_t scratch_device_ptr(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace sf
