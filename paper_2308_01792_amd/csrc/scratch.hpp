// Allocation-free scratch (scratch.hip).
#pragma once
#include <stdint.h>

namespace ht {

// Capacity in FP64 values (4 MiB per GPU) and the highest device index
// served.
enum : int64_t { kNoAllocScratch = int64_t(1) << 19 };
enum { kNoAllocDevices = 64 };

// Device address of the calling thread's current device's scratch array
// (looked up on the first call per device).  Throws Error on HIP failure.
double* noalloc_scratch();

}  // namespace ht
