// Storage codec for population buffers. The stored quantity is already the deviation
// g_i = f_i - w_i rho0 (the delta-rho form of the equilibrium, which the paper adopts to
// limit round-off), so FP16/BF16 storage keeps only the small part of f. All arithmetic is
// FP32; stores round to nearest even.
#pragma once
#include <hip/hip_runtime.h>

namespace lbm {

// Population planes are streamed: every element is read once and written once per step,
// so their loads and stores carry the nontemporal hint (load_cached is the plain load).
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void stream_store(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

template <typename S>
struct Codec;

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// kMixedFma: the arithmetic may take loaded values straight into mixed-precision FMAs
// (v_fma_mix_f32 reads FP16 operands; there is no such form for BF16).
template <>
struct Codec<float> {
  static constexpr bool kMixedFma = false;
  static __device__ __forceinline__ float load_cached(const float* p) { return *p; }
  static __device__ __forceinline__ float load(const float* p) { return stream_load(p); }
  static __device__ __forceinline__ void store(float* p, float v) { stream_store(p, v); }
};

template <>
struct Codec<_Float16> {
  static constexpr bool kMixedFma = true;
  static __device__ __forceinline__ float load_cached(const _Float16* p) { return static_cast<float>(*p); }
  static __device__ __forceinline__ float load(const _Float16* p) { return static_cast<float>(stream_load(p)); }
  // fptrunc float -> half rounds to nearest even (default rounding mode).
  static __device__ __forceinline__ void store(_Float16* p, float v) { stream_store(p, static_cast<_Float16>(v)); }
  // Two values rounded by one packed conversion: a in the low half, b in the high half.
  // (Taken apart as a 32-bit word: element access on the converted vector is avoided.)
  static __device__ __forceinline__ unsigned encode2(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, f16x2));
  }
};

template <>
struct Codec<__bf16> {
  static constexpr bool kMixedFma = false;
  static __device__ __forceinline__ float load_cached(const __bf16* p) { return static_cast<float>(*p); }
  static __device__ __forceinline__ float load(const __bf16* p) { return static_cast<float>(stream_load(p)); }
  // fptrunc float -> bfloat rounds to nearest even.
  static __device__ __forceinline__ void store(__bf16* p, float v) { stream_store(p, static_cast<__bf16>(v)); }
  static __device__ __forceinline__ unsigned encode2(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, bf16x2));
  }
};

}  // namespace lbm
