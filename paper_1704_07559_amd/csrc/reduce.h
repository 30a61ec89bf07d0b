// Deterministic FP64 block reduction of kReduceVals values per thread. Slot 6 is reduced
// with max, every other slot with +. The order of every addition is fixed by the launch
// shape, so repeated runs give identical bits.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"

namespace lbm {

__device__ __forceinline__ double combine(int k, double a, double b) { return k == 6 ? fmax(a, b) : a + b; }

// Block of 256 threads (4 waves of 64). Thread 0 writes partials[blockIdx.x * 8 + k].
__device__ __forceinline__ void block_reduce_store(double (&v)[kReduceVals], double* partials) {
  __shared__ double sh[4][kReduceVals];
#pragma unroll
  for (int k = 0; k < kReduceVals; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] = combine(k, v[k], __shfl_xor(v[k], off, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kReduceVals; ++k) sh[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kReduceVals; ++k) {
      double a = sh[0][k];
      for (int w = 1; w < 4; ++w) a = combine(k, a, sh[w][k]);
      partials[blockIdx.x * kReduceVals + k] = a;
    }
  }
}

}  // namespace lbm
