// Second pass of the deterministic FP64 reductions: slot k of the result is the fold of
// slot k over the per-block partials. Thread t folds partials t, t+256, t+512, ... in
// order, then the 256 thread results are folded by the fixed block tree of reduce.h.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"
#include "reduce.h"

namespace lbm {

// rho0 > 0: slot 6 holds the largest |j|^2 and becomes max |u| = sqrt(max |j|^2) / rho0 (one
// square root and one division instead of one per node; both are correctly rounded and
// monotone, so this is the maximum of the per-node values bit for bit).
__global__ __launch_bounds__(256) void reduce_final_kernel(const double* __restrict__ partials, int nblocks,
                                                           double* __restrict__ out, double rho0) {
  double v[kReduceVals];
#pragma unroll
  for (int k = 0; k < kReduceVals; ++k) v[k] = 0.0;  // max slot: |j|^2 >= 0
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kReduceVals; ++k) v[k] = combine(k, v[k], partials[b * kReduceVals + k]);
  }
  block_reduce_store(v, out);  // gridDim.x == 1: thread 0 writes out[0..7]
  if (threadIdx.x == 0 && rho0 > 0.0) out[6] = sqrt(out[6]) / rho0;
}

hipError_t launch_reduce_final(const double* partials, int nblocks, double* out, hipStream_t st, double rho0) {
  hipLaunchKernelGGL(reduce_final_kernel, dim3(1), dim3(256), 0, st, partials, nblocks, out, rho0);
  return hipGetLastError();
}

}  // namespace lbm
