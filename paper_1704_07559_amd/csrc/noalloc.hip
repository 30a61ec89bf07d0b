// Device scratch for the allocation-free entry point (lbm_adjoint_steps_noalloc): a
// file-scope array that every GPU the library runs on holds from module load until the
// process ends. Host code never passes the array's name to a kernel or a copy (on the host it
// is only a stand-in for the symbol): each device's own address is looked up once with
// hipGetSymbolAddress, with that device current, and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "launch.h"

static __device__ __align__(256) float scratch[lbm::kNoAllocScratchBytes / sizeof(float)];

namespace lbm {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(hipStream_t stream, void** out) {
  *out = nullptr;
  hipDevice_t dev = 0;
  hipError_t e = hipStreamGetDevice(stream, &dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t restore = (cur != dev) ? hipSetDevice(cur) : hipSuccess;
    if (e != hipSuccess) return e;
    if (restore != hipSuccess) return restore;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace lbm
