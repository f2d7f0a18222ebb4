// Device probes (k_probe.hip): machine constants measured on the current
// device.  Each call allocates its own buffers, runs on stream st and
// synchronises it.
#pragma once

#include <hip/hip_runtime.h>

namespace sf {

// Read + write bytes per second of a 1 GiB -> 1 GiB stream copy, in GB/s.
hipError_t probe_copy(int cus, hipStream_t st, double* gbps);
// One-way hop of a published value (us) between two workgroups on one XCD
// and across XCDs; -1 where no pair of that kind was placed or a poll gave up.
hipError_t probe_hop(hipStream_t st, double* same_us, double* cross_us);
// Random single-value FP64 gathers per second (2^20-entry vector, 5e7 gathers).
hipError_t probe_gather(int cus, hipStream_t st, double* per_s);

}  // namespace sf
