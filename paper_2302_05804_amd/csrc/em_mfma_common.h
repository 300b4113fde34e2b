// em_mfma_common.h -- helpers shared by the matrix-core kernels of libem.so.
#pragma once

#include <hip/hip_runtime.h>

namespace em {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// Row pitch (bf16 elements) of an LDS plane holding `cols` columns: rows stay
// 16-byte aligned and the pitch is an odd number of 16-byte chunks.
__host__ __device__ constexpr int mf_pitch(int cols) {
  return (((cols + 7) / 8) % 2 == 1) ? ((cols + 7) / 8) * 8 : ((cols + 7) / 8) * 8 + 8;
}

__device__ inline unsigned short bf16_bits(__bf16 v) { return __builtin_bit_cast(unsigned short, v); }

// v = hi + lo with hi = bf16(v), lo = bf16(v - hi) (round to nearest even).
__device__ inline void split_bf16(float v, unsigned short& hi, unsigned short& lo) {
  const __bf16 h = (__bf16)v;
  const float rest = v - (float)h;
  hi = bf16_bits(h);
  lo = bf16_bits((__bf16)rest);
}

__device__ inline float mf_update_value(float xo, float Bv, float Dn) {
  if (xo == 0.f) return 0.f;
  if (Dn == 0.f) return xo;
  const float q = fmaxf(Bv, 0.f) / Dn;
  return xo * q;
}

}  // namespace em
