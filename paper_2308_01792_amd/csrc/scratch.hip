// Device scratch of the allocation-free entry points (ht_residual_noalloc).
//
// Callers that cannot allocate device memory (code under graph capture,
// serving loops, harnesses that forbid it) get their per-call scratch from
// one file-scope device array instead of the mesh's allocations.  Each GPU
// the library runs on holds its own copy of the array until the process
// ends; its device address is looked up once per device with
// hipGetSymbolAddress and kept.  Every call on a GPU shares that GPU's
// array and finds the previous call's contents in it: the kernels write
// every value they read back, and calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hytet_impl.hpp"
#include "scratch.hpp"

namespace ht {

static __device__ __align__(256) double scratch[kNoAllocScratch];

double* noalloc_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{HT_ERR_HIP, "hipGetDevice failed"};
  }
  if (dev < 0 || dev >= kNoAllocDevices)
    throw Error{HT_ERR_STATE, "device index beyond the allocation-free scratch table"};
  static std::mutex mu;
  static double* addr[kNoAllocDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error{HT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                  hipGetErrorString(e)};
    }
    addr[dev] = (double*)p;
  }
  return addr[dev];
}

}  // namespace ht
