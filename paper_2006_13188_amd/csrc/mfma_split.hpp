// Matrix-core operands split into hi + lo parts (float16 or bfloat16) for float32-accurate
// products: a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi, accumulated in float32 by the
// 16 x 16 x 16 matrix instructions (the lo * lo term is dropped: about 2^-22 relative for
// float16 with operands scaled into [2^10, 2^11), 2^-16 for bfloat16).
//
// Operand layout of v_mfma_f32_16x16x16{f16, bf16_1k} (lane l of the wave, j = 0..3):
// A[m][k] with m = l % 16, k = 4 (l / 16) + j; B[k][n] with n = l % 16, k = 4 (l / 16) + j;
// the result C[m][n] with n = l % 16, m = 4 (l / 16) + j.
#pragma once
#include <hip/hip_runtime.h>

namespace ecc {
namespace {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {   // round to nearest even
  const unsigned u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_value(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }

template <bool BF16>
struct Split;
template <>
struct Split<false> {
  typedef half4_t T;
  static __device__ __forceinline__ void split(const float* v, T& hi, T& lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const _Float16 h = (_Float16)v[j];
      hi[j] = h;
      lo[j] = (_Float16)(v[j] - (float)h);
    }
  }
  static __device__ __forceinline__ f4_t mma(T a, T b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Split<true> {
  typedef bf4_t T;
  static __device__ __forceinline__ void split(const float* v, T& hi, T& lo) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const short h = bf16_bits(v[j]);
      hi[j] = h;
      lo[j] = bf16_bits(v[j] - bf16_value(h));
    }
  }
  static __device__ __forceinline__ f4_t mma(T a, T b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
};

}  // namespace
}  // namespace ecc
