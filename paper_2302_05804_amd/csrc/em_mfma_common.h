// em_mfma_common.h -- helpers shared by the matrix-core kernels of libem.so.
#pragma once

#include <hip/hip_runtime.h>

namespace em {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// Row pitch (bf16 elements) of an LDS plane holding `cols` columns whose
// 16-byte fragments are read by lanes i = 0..15 at rows base + row_stride * i
// and by the next lane group one chunk to the right.  A ds_read_b128 serves
// lanes {0-7, 16-23} (and the matching groups) together across 64 banks; the
// sixteen 16-byte pieces are conflict-free when row_stride * pitch, counted in
// 16-byte chunks, is 2 mod 4 (measured on gfx950: 22 chunks conflict-free, 21,
// 23 and 25 chunks four extra cycles per read, 24 chunks twelve).
__host__ __device__ constexpr int mf_pitch(int cols, int row_stride = 1) {
  int chunks = (cols + 7) / 8;
  while ((row_stride * chunks) % 4 != 2) ++chunks;
  return chunks * 8;
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
