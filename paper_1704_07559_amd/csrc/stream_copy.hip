// STREAM-style copy: the achievable HBM bandwidth on this device for a pure streaming
// pattern (one read and one write per byte, 16-byte nontemporal accesses, every address
// touched once). The benchmark reports it next to the step kernel, whose roofline is the
// same two streams per population.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "launch.h"

namespace lbm {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void stream_copy_kernel(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                          size_t n4) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  const size_t n4 = bytes / 16;
  if (n4 == 0) return hipSuccess;
  const size_t blocks = (n4 + 255) / 256;
  if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
  // 5 blocks per CU instead of 8: the copy's own best (6.73 against 6.63 TB/s for 1 GiB; 6 blocks
  // 6.69, 4 blocks 6.38), so that it stays the ceiling the step is compared with
  hipLaunchKernelGGL(stream_copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), lds_cap_bytes(5, 0), st,
                     static_cast<const v4f*>(src), static_cast<v4f*>(dst), n4);
  return hipGetLastError();
}

}  // namespace lbm
