// Compile-time loop helper: the body receives std::integral_constant<int, I> so table
// lookups with I fold to constants and zero coefficients drop out with `if constexpr`.
#pragma once
#include <utility>

namespace lbm {

template <class F, int... I>
__host__ __device__ __forceinline__ constexpr void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}

template <int N, class F>
__host__ __device__ __forceinline__ constexpr void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// acc + C*x with the integer coefficient C known at compile time.
template <int C>
__device__ __forceinline__ float acc_int(float acc, float x) {
  if constexpr (C == 0) return acc;
  else if constexpr (C == 1) return acc + x;
  else if constexpr (C == -1) return acc - x;
  else return __builtin_fmaf(static_cast<float>(C), x, acc);
}

}  // namespace lbm
