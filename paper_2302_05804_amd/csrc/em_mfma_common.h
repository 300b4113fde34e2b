// em_mfma_common.h -- operand encodings and tile staging shared by the
// matrix-core kernels of libem.so (em_mfma.hip, sr = 1; em_mfma2.hip, sr = 2).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "em.h"
#include "em_device.h"

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

// Start copying NTF Toeplitz fragments (64 lanes x 16 bytes each) of one
// frame's table into an LDS buffer: buffer fragment f comes from table
// fragment idx(f).  The NW waves of the workgroup share the fragments round
// robin; each lane moves its own 16 bytes with global_load_lds_dwordx4, whose
// destination is the wave-uniform base plus 16 bytes per lane (the fragment's
// lane order).  Completion: s_waitcnt in each wave, then a barrier.
template <int NTF, int NW, class Frag, class Idx>
__device__ inline void stage_frags(const Frag* __restrict__ tab_t, Idx idx, void* dst_v) {
  Frag* dst = static_cast<Frag*>(dst_v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int f = w; f < NTF; f += NW) {
    const Frag* src = tab_t + idx(f) * 64 + lane;
    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src),
                                     (__attribute__((address_space(3))) void*)(dst + f * 64), 16,
                                     0, 0);
  }
}

// Wait for this wave's fragment copies, then for every wave of the workgroup.
__device__ inline void frags_landed() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
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
// call it (one barrier inside); `redf` holds NT/64 floats of LDS.  Unscaled
// encodings load SB pixel pairs per thread at a time (SB = 0: one pair, stored
// before the next is loaded).
template <int PREC, int ROWS, int COLS, int PITCH, int NT, int SB = 8>
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
  if constexpr (!Prec<PREC>::SCALED && SB == 0) {
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
  } else if constexpr (!Prec<PREC>::SCALED) {
    // batches of SB pixel pairs per thread: the batch's loads read clamped
    // addresses inside the image (values outside it replaced by 0), so they
    // carry no branches and are in flight together, one wait per batch
    constexpr int NPT = (NE + NT - 1) / NT;
#pragma unroll
    for (int k0 = 0; k0 < NPT; k0 += SB) {
      float v[SB][2];
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const int e = threadIdx.x + (k0 + k) * NT;
        const int row = e / HALF, cp = e - row * HALF;
        const int gy = r0 + row, gx = q0 + 2 * cp;
        const bool iny = e < NE && gy >= 0 && gy < H;
        const float* rp = src + (int64_t)min(max(gy, 0), H - 1) * W;
        const float a0 = rp[min(max(gx, 0), W - 1)];
        const float a1 = rp[min(max(gx + 1, 0), W - 1)];
        v[k][0] = (iny && gx >= 0 && gx < W) ? a0 : 0.f;
        v[k][1] = (iny && gx + 1 >= 0 && gx + 1 < W) ? a1 : 0.f;
      }
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const int e = threadIdx.x + (k0 + k) * NT;
        if (e < NE) {
          const int row = e / HALF, cp = e - row * HALF;
          const int o = row * PITCH + 2 * cp;
          unsigned short h0, l0, h1, l1;
          split_bf16(v[k][0], h0, l0);
          split_bf16(v[k][1], h1, l1);
          *reinterpret_cast<unsigned int*>(&sh[0][o]) = (unsigned int)h0 | ((unsigned int)h1 << 16);
          if constexpr (Prec<PREC>::NA == 2)
            *reinterpret_cast<unsigned int*>(&sh[1][o]) = (unsigned int)l0 | ((unsigned int)l1 << 16);
        }
      }
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

// Output position of accumulator element (b, q, v) of a wave whose block
// (0, 0) starts at row kb, column lb; rows of the blocks are rs apart (2 for the
// parity-split outputs of the sr = 2 adjoint).
struct BlockPos {
  int kb, lb, rs;
  __device__ int row(int b, int v) const {
    return kb + rs * (16 * b + 4 * ((threadIdx.x & 63) >> 4) + v);
  }
  __device__ int col(int q) const { return lb + 16 * q + (threadIdx.x & 15); }
};

// Forward epilogue of one frame: out = u * m (m = F_t x, unscaled by 2^unscale)
// or out = m when u is NULL, plus the FP64 partial of u (y - m)^2 when y is
// given (WITH_Y).  Every load is issued before any store (addresses clamped
// into the image; clamped values are never used), so one wait covers them all.
template <int BR, int BC, bool WITH_Y>
__device__ inline double forward_epilogue_w(const f32x4 (&acc)[BR][BC], int unscale,
                                            const BlockPos& P, int H, int W,
                                            const float* __restrict__ ut,
                                            const float* __restrict__ yt,
                                            float* __restrict__ ot) {
  float uu[BR][BC][4], yy[BR][BC][4];
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int off = min(P.row(b, v), H - 1) * W + min(P.col(q), W - 1);
        uu[b][q][v] = ut[off];
        if constexpr (WITH_Y) yy[b][q][v] = yt[off];
      }
  double llp = 0.0;
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = P.row(b, v), l = P.col(q);
        if (k < H && l < W) {
          const float m = ldexpf(acc[b][q][v], unscale);
          const float u = uu[b][q][v];
          if (ot) ot[k * W + l] = u * m;
          if constexpr (WITH_Y) {
            if (u > 0.f) {
              const double d = (double)yy[b][q][v] - (double)m;
              llp += (double)u * d * d;
            }
          }
        }
      }
  return llp;
}

// Forward epilogue under Student-t noise: with m = F_t x and the E-step weight
// w = (nu + 1) / (nu + u (y - m)^2) of each observed pixel, out = u w m and
// out_y = u w y (0 where u = 0); with `ll`, the FP64 partial of
// (nu + 1) ln(1 + u (y - m)^2 / nu) - lcst.  Loads first, as below.
template <int BR, int BC>
__device__ inline double forward_epilogue_t(const f32x4 (&acc)[BR][BC], int unscale,
                                            const BlockPos& P, int H, int W,
                                            const float* __restrict__ ut,
                                            const float* __restrict__ yt, float* __restrict__ ot,
                                            float* __restrict__ oyt, float nu, double lcst,
                                            bool ll) {
  // two halves of the block rows, each with its loads issued first: half the
  // registers of loading u and y for every output at once
  constexpr int BH = (BR + 1) / 2;
  const float nu1 = nu + 1.f;
  double llp = 0.0;
#pragma unroll
  for (int h = 0; h < BR; h += BH) {
    float uu[BH][BC][4], yy[BH][BC][4];
#pragma unroll
    for (int bb = 0; bb < BH; ++bb)
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int b = min(h + bb, BR - 1);
          const int off = min(P.row(b, v), H - 1) * W + min(P.col(q), W - 1);
          uu[bb][q][v] = ut[off];
          yy[bb][q][v] = yt[off];
        }
#pragma unroll
    for (int bb = 0; bb < BH; ++bb) {
      const int b = h + bb;
      if (b >= BR) break;
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = P.row(b, v), l = P.col(q);
          if (k < H && l < W) {
            const float m = ldexpf(acc[b][q][v], unscale);
            const float u = uu[bb][q][v];
            float ro = 0.f, ryo = 0.f;
            if (u > 0.f) {
              const float y = yy[bb][q][v];
              const float d = y - m;
              const float w = nu1 / (nu + u * d * d);
              ro = (u * w) * m;
              ryo = (u * w) * y;
              if (ll) {
                const double dd = (double)y - (double)m;
                llp += ((double)nu + 1.0) * log1p((double)u * dd * dd / (double)nu) - lcst;
              }
            }
            ot[k * W + l] = ro;
            oyt[k * W + l] = ryo;
          }
        }
    }
  }
  return llp;
}

// Copy of a frame's u tile (TH x TW floats from (k0, l0), rows and columns clamped
// into the frame, which is a multiple of 4 wide) into LDS, 1 KB per direct
// global-to-LDS instruction, spread over tap classes 1..13 of the frame (class
// 0's barrier separates it from the previous frame's epilogue reads).
struct UPre {
  const float* ut;   // frame base of u, or nullptr (no copy)
  float* ub;         // LDS destination
  int k0, l0, H, W;
};
// Returns the number of copies this wave issued (at most 2).
template <int TH, int TW, int NW>
__device__ inline int issue_u_tile(const UPre& u, int r) {
  static_assert(256 % TW == 0, "a 1 KB chunk holds whole tile rows");
  constexpr int NCH = TH * TW / 256;         // 1 KB chunks of the tile
  constexpr int CPC = (NCH + 12) / 13;       // chunks per class, classes 1..13
  static_assert(CPC <= 2 * NW, "at most two copies per wave and class");
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (u.ut == nullptr || r < 1 || r > 13) return 0;
  const int end = min(r * CPC, NCH);
  int issued = 0;
  for (int ch = (r - 1) * CPC + w; ch < end; ch += NW) {
    const int e = ch * 256 + 4 * lane;
    const int gy = min(u.k0 + e / TW, u.H - 1), gx = min(u.l0 + e % TW, u.W - 4);
    __builtin_amdgcn_global_load_lds(
        (__attribute__((address_space(1))) void*)(u.ut + (int64_t)gy * u.W + gx),
        (__attribute__((address_space(3))) void*)(u.ub + ch * 256), 16, 0, 0);
    ++issued;
  }
  return issued;
}

// Forward epilogue with u already in LDS (ub: the tile's TH x TW weights, row-major
// from (k0, l0)): out = u * m.
template <int BR, int BC, int TW>
__device__ inline void forward_epilogue_ul(const f32x4 (&acc)[BR][BC], int unscale,
                                           const BlockPos& P, int H, int W, int k0, int l0,
                                           const float* ub, float* __restrict__ ot) {
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = P.row(b, v), l = P.col(q);
        if (k < H && l < W) {
          const float m = ldexpf(acc[b][q][v], unscale);
          ot[k * W + l] = ub[(k - k0) * TW + (l - l0)] * m;
        }
      }
}

// Forward epilogues that write r = u m as binary16 into an r16 plane (rows of
// `pitch` halves, frame pixel (k, l) at row k + off, column l + off), scaled
// by 2^e: the FP32 product u m, then the exact power-of-two scale, then one
// rounding to binary16 (the encoding the adjoint's staging used to apply).
struct R16Out {
  unsigned short* plane;
  int pitch, off, e;
  __device__ void put(int k, int l, float r) const {
    plane[(int64_t)(k + off) * pitch + (l + off)] = f16_bits((_Float16)ldexpf(r, e));
  }
};

// u from LDS (ub: the tile's TH x TW weights from (k0, l0)), as forward_epilogue_ul.
template <int BR, int BC, int TW>
__device__ inline void forward_epilogue_ul16(const f32x4 (&acc)[BR][BC], int unscale,
                                             const BlockPos& P, int H, int W, int k0, int l0,
                                             const float* ub, const R16Out& o) {
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = P.row(b, v), l = P.col(q);
        if (k < H && l < W) {
          const float m = ldexpf(acc[b][q][v], unscale);
          o.put(k, l, ub[(k - k0) * TW + (l - l0)] * m);
        }
      }
}

// u (and y, for the loglik partial of u (y - m)^2) from HBM, loads first, as
// forward_epilogue_w.
template <int BR, int BC, bool WITH_Y>
__device__ inline double forward_epilogue_w16(const f32x4 (&acc)[BR][BC], int unscale,
                                              const BlockPos& P, int H, int W,
                                              const float* __restrict__ ut,
                                              const float* __restrict__ yt, const R16Out& o) {
  float uu[BR][BC][4], yy[BR][BC][4];
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int off = min(P.row(b, v), H - 1) * W + min(P.col(q), W - 1);
        uu[b][q][v] = ut[off];
        if constexpr (WITH_Y) yy[b][q][v] = yt[off];
      }
  double llp = 0.0;
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = P.row(b, v), l = P.col(q);
        if (k < H && l < W) {
          const float m = ldexpf(acc[b][q][v], unscale);
          const float u = uu[b][q][v];
          o.put(k, l, u * m);
          if constexpr (WITH_Y) {
            if (u > 0.f) {
              const double d = (double)yy[b][q][v] - (double)m;
              llp += (double)u * d * d;
            }
          }
        }
      }
  return llp;
}

template <int BR, int BC>
__device__ inline double forward_epilogue(const f32x4 (&acc)[BR][BC], int unscale,
                                          const BlockPos& P, int H, int W,
                                          const float* __restrict__ ut,
                                          const float* __restrict__ yt, float* __restrict__ ot) {
  if (ut == nullptr) {
#pragma unroll
    for (int b = 0; b < BR; ++b)
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = P.row(b, v), l = P.col(q);
          if (k < H && l < W) ot[k * W + l] = ldexpf(acc[b][q][v], unscale);
        }
    return 0.0;
  }
  return yt ? forward_epilogue_w<BR, BC, true>(acc, unscale, P, H, W, ut, yt, ot)
            : forward_epilogue_w<BR, BC, false>(acc, unscale, P, H, W, ut, yt, ot);
}

// Adjoint epilogue: Dn = acc.  Fused update of Eq. (2) (x <- x max(B,0)/Dn,
// FP64 partials of |x_new - x|^2 and |x|^2) or a store into the partial plane.
// Loads first, as in forward_epilogue.
template <int BR, int BC>
__device__ inline void adjoint_epilogue(const f32x4 (&acc)[BR][BC], const BlockPos& P, int H,
                                        int W, bool fused, float* __restrict__ x,
                                        const float* __restrict__ B, float* __restrict__ plane,
                                        double& dsq, double& xsq) {
  if (!fused) {
#pragma unroll
    for (int b = 0; b < BR; ++b)
#pragma unroll
      for (int q = 0; q < BC; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = P.row(b, v), l = P.col(q);
          if (k < H && l < W) plane[k * W + l] = acc[b][q][v];
        }
    return;
  }
  float xo[BR][BC][4], bv[BR][BC][4];
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int off = min(P.row(b, v), H - 1) * W + min(P.col(q), W - 1);
        xo[b][q][v] = x[off];
        bv[b][q][v] = B[off];
      }
#pragma unroll
  for (int b = 0; b < BR; ++b)
#pragma unroll
    for (int q = 0; q < BC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = P.row(b, v), l = P.col(q);
        if (k < H && l < W) {
          const float xn = em_update_value(xo[b][q][v], bv[b][q][v], acc[b][q][v]);
          x[k * W + l] = xn;
          const double d = (double)xn - (double)xo[b][q][v];
          dsq += d * d;
          xsq += (double)xo[b][q][v] * (double)xo[b][q][v];
        }
      }
}

}  // namespace em
