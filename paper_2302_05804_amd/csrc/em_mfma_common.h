// em_mfma_common.h -- operand encodings and tile staging shared by the
// matrix-core kernels of libem.so (em_mfma.hip, sr = 1; em_mfma2.hip, sr = 2).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "em.h"

namespace em {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// Row pitch (16-bit elements) of an LDS plane holding `cols` columns whose
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
__device__ inline unsigned short f16_bits(_Float16 v) { return __builtin_bit_cast(unsigned short, v); }

// v = hi + lo with hi = bf16(v), lo = bf16(v - hi) (round to nearest even).
__device__ inline void split_bf16(float v, unsigned short& hi, unsigned short& lo) {
  const __bf16 h = (__bf16)v;
  const float rest = v - (float)h;
  hi = bf16_bits(h);
  lo = bf16_bits((__bf16)rest);
}

// Same split in binary16 (v already scaled into the binary16 range).
__device__ inline void split_f16(float v, unsigned short& hi, unsigned short& lo) {
  const _Float16 h = (_Float16)v;
  const float rest = v - (float)h;
  hi = f16_bits(h);
  lo = f16_bits((_Float16)rest);
}

// Power-of-two scale 2^e that brings a largest magnitude `mx` into
// [2^14, 2^15): binary16 then keeps 11 significant bits for every value down
// to 2^-29 of the largest and cannot overflow.  0 (all zero) and non-finite
// maxima get e = 0 (non-finite values then propagate as they would in FP32).
__host__ __device__ inline int f16_scale_exp(float mx) {
  if (!(mx > 0.f) || !(mx < INFINITY)) return 0;
  int e;
  (void)frexpf(mx, &e);   // mx = m 2^e, m in [0.5, 1)
  return 15 - e;
}

// Operand encodings of the matrix-core forms (template argument PREC of the
// kernels).  A is the image operand (staged in LDS), B the Toeplitz PSF
// operand (pre-built tables); product s multiplies A part pa(s) by B part pb(s)
// and every product accumulates into the same FP32 accumulator.
//   EM_BF16_SPLIT: A and B split into bf16 hi + lo; hi.hi + lo.hi + hi.lo
//                  (the lo.lo term, ~2^-16 relative, is dropped).
//   EM_BF16:       plain bf16 operands, one product (ablation).
//   EM_FP16_SPLIT: A binary16, one part, scaled by a power of two per staged
//                  tile; B binary16 hi + lo, scaled by a power of two per frame;
//                  A.hi + A.lo.  The epilogue removes both scales exactly.
template <int PREC>
struct Prec;

template <>
struct Prec<EM_BF16_SPLIT> {
  using frag = bf16x8;
  static constexpr int NA = 2, NB = 2, NP = 3;
  static constexpr bool SCALED = false;
  __device__ static constexpr int pa(int s) { return s == 1 ? 1 : 0; }
  __device__ static constexpr int pb(int s) { return s == 2 ? 1 : 0; }
  __device__ static inline f32x4 mma(const frag& a, const frag& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Prec<EM_BF16> {
  using frag = bf16x8;
  static constexpr int NA = 1, NB = 1, NP = 1;
  static constexpr bool SCALED = false;
  __device__ static constexpr int pa(int) { return 0; }
  __device__ static constexpr int pb(int) { return 0; }
  __device__ static inline f32x4 mma(const frag& a, const frag& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Prec<EM_FP16_SPLIT> {
  using frag = f16x8;
  static constexpr int NA = 1, NB = 2, NP = 2;
  static constexpr bool SCALED = true;
  __device__ static constexpr int pa(int) { return 0; }
  __device__ static constexpr int pb(int s) { return s; }
  __device__ static inline f32x4 mma(const frag& a, const frag& b, const f32x4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// Table entry of PSF value gv (already multiplied by the frame's scale for
// scaled forms), part s.
template <int PREC>
__device__ inline unsigned short table_part(float gv, int s) {
  unsigned short hi, lo;
  if constexpr (PREC == EM_FP16_SPLIT) split_f16(gv, hi, lo);
  else split_bf16(gv, hi, lo);
  return s == 0 ? hi : lo;
}

__device__ inline float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// Stage an FP32 image tile (rows [r0, r0 + ROWS), cols [q0, q0 + COLS), zero
// outside [0,H) x [0,W)) into the LDS planes of encoding PREC, row pitch PITCH.
// Returns the tile's scale exponent (0 for unscaled encodings); every thread of
// the block gets the same value.  For scaled encodings the whole block must
// call it (one barrier inside); `redf` holds NT/64 floats of LDS.
template <int PREC, int ROWS, int COLS, int PITCH, int NT>
__device__ inline int stage_tile(const float* __restrict__ src, int H, int W, int r0, int q0,
                                 unsigned short (*sh)[ROWS * PITCH], float* redf) {
  constexpr int HALF = COLS / 2;
  constexpr int NE = ROWS * HALF;
  auto load2 = [&](int e, float& v0, float& v1) {
    const int row = e / HALF, cp = e - row * HALF;
    const int gy = r0 + row, gx = q0 + 2 * cp;
    v0 = 0.f;
    v1 = 0.f;
    if (gy >= 0 && gy < H) {
      const float* rp = src + (int64_t)gy * W;
      if (gx >= 0 && gx < W) v0 = rp[gx];
      if (gx + 1 >= 0 && gx + 1 < W) v1 = rp[gx + 1];
    }
    return row * PITCH + 2 * cp;
  };
  if constexpr (!Prec<PREC>::SCALED) {
    for (int e = threadIdx.x; e < NE; e += NT) {
      float v0, v1;
      const int o = load2(e, v0, v1);
      unsigned short h0, l0, h1, l1;
      split_bf16(v0, h0, l0);
      split_bf16(v1, h1, l1);
      *reinterpret_cast<unsigned int*>(&sh[0][o]) = (unsigned int)h0 | ((unsigned int)h1 << 16);
      if constexpr (Prec<PREC>::NA == 2)
        *reinterpret_cast<unsigned int*>(&sh[1][o]) = (unsigned int)l0 | ((unsigned int)l1 << 16);
    }
    return 0;
  } else {
    // all loads first (kept in registers), then the tile maximum, then the
    // scaled binary16 values
    constexpr int NPT = (NE + NT - 1) / NT;
    float v[NPT][2];
    float mx = 0.f;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int e = threadIdx.x + k * NT;
      v[k][0] = 0.f;
      v[k][1] = 0.f;
      if (e < NE) (void)load2(e, v[k][0], v[k][1]);
      mx = fmaxf(mx, fmaxf(fabsf(v[k][0]), fabsf(v[k][1])));
    }
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = mx;
    __syncthreads();
    float bm = redf[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) bm = fmaxf(bm, redf[i]);
    const int ex = f16_scale_exp(bm);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int e = threadIdx.x + k * NT;
      if (e < NE) {
        const int row = e / HALF, cp = e - row * HALF;
        const unsigned short h0 = f16_bits((_Float16)ldexpf(v[k][0], ex));
        const unsigned short h1 = f16_bits((_Float16)ldexpf(v[k][1], ex));
        *reinterpret_cast<unsigned int*>(&sh[0][row * PITCH + 2 * cp]) =
            (unsigned int)h0 | ((unsigned int)h1 << 16);
      }
    }
    return ex;
  }
}

__device__ inline float mf_update_value(float xo, float Bv, float Dn) {
  if (xo == 0.f) return 0.f;
  if (Dn == 0.f) return xo;
  const float q = fmaxf(Bv, 0.f) / Dn;
  return xo * q;
}

}  // namespace em
