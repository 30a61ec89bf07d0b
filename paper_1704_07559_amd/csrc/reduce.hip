// Second pass of the deterministic FP64 reductions: slot k of the result is the fold of
// slot k over the per-block partials. Thread t folds partials t, t+256, t+512, ... in
// order, then the 256 thread results are folded by the fixed block tree of reduce.h.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {

__global__ __launch_bounds__(256) void reduce_final_kernel(const double* __restrict__ partials, int nblocks,
                                                           double* __restrict__ out) {
  double v[kReduceVals];
#pragma unroll
  for (int k = 0; k < kReduceVals; ++k) v[k] = 0.0;  // max slot: |u| >= 0
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kReduceVals; ++k) v[k] = combine(k, v[k], partials[b * kReduceVals + k]);
  }
  block_reduce_store(v, out);  // gridDim.x == 1: writes out[0..7]
}

hipError_t launch_reduce_final(const double* partials, int nblocks, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, out);
  return hipGetLastError();
}

}  // namespace lbm
