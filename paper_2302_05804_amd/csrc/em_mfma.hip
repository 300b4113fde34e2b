// em_mfma.hip -- BF16 matrix-core (MFMA) form of the two convolutions of one
// EM iteration (arXiv:2302.05804, Sec. 2, Eqs. (1)-(2)), sr = 1.
//
// Both directions are the same 2-D correlation core
//     out[k][l] = sum_{a,b} g[a][b] in[k - c + a][l - c + b]
// with g = f flipped by 180 degrees for the forward model (f * x) and g = f for
// the adjoint F^T r.  For one kernel row a the sum over b is a 1-D correlation,
// i.e. a product with a banded Toeplitz matrix:
//     O(16 x 16) += X_a(16 x 64) . U_a(64 x 16),
//     X_a[i][p] = in[k0 + i - c + a][l0 - c + p],   U_a[p][j] = g[a][p - j]
// (zero outside 0 <= p - j < K).  Each product is two
// v_mfma_f32_16x16x32_bf16 steps (p in [0,32) and [32,64)); 43 of the 64
// p-values of a column of U_a are non-zero.
//
// Precision: operands are split into bf16 hi + lo parts (v = hi + lo, with
// lo = bf16(v - hi)) and each product is formed as hi.hi + lo.hi + hi.lo with
// FP32 accumulation in the matrix core (the lo.lo term, ~2^-16 relative, is
// dropped).  NS = 1 keeps only hi.hi (plain bf16, for comparison).
//
// Data movement (per workgroup of 4 waves, 128 x 128 outputs, each wave 64 x 64
// = 4 x 4 blocks of 16 x 16):
//  * the input tile (128 + K - 1 rows, 176 columns) is stored in LDS as two
//    bf16 planes (hi, lo), row-major, row pitch 368 bytes (an odd multiple of 16
//    bytes, so 16-byte fragment reads of consecutive rows spread over banks);
//  * taps are grouped in classes a = r + 16 m: the A fragment of rows
//    r + 16 rho + i then serves block rows beta = rho - m for every m of the
//    class, so one LDS read feeds up to 3 row blocks (and 2 column blocks);
//  * the Toeplitz fragments U_a (hi, lo) are pre-built per frame in the lane
//    order of the MFMA B operand and read from global memory (L2-resident).
#include "em_device.h"
#include "em_internal.h"

namespace em {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int MF_BR = 4, MF_BC = 4;          // 16x16 blocks per wave (rows, cols)
constexpr int MF_TH = 128, MF_TW = 128;      // outputs per workgroup
constexpr int MF_COLS = MF_TW + 48;          // LDS columns read by fragments
constexpr int MF_PITCH = 184;                // bf16 per LDS row (368 bytes)
constexpr int MF_NT = 256;

__device__ inline unsigned short bf16_bits(__bf16 v) { return __builtin_bit_cast(unsigned short, v); }

// v = hi + lo with hi = bf16(v), lo = bf16(v - hi) (round to nearest even).
__device__ inline void split_bf16(float v, unsigned short& hi, unsigned short& lo) {
  const __bf16 h = (__bf16)v;
  const float rest = v - (float)h;
  hi = bf16_bits(h);
  lo = bf16_bits((__bf16)rest);
}

// Stage an input tile (FP32 image, rows [r0, r0 + ROWS), cols [q0, q0 + MF_COLS),
// zero outside [0,H) x [0,W)) into the hi / lo LDS planes.
template <int ROWS>
__device__ inline void stage_tile(const float* __restrict__ src, int H, int W, int r0, int q0,
                                  unsigned short* sh_hi, unsigned short* sh_lo) {
  constexpr int HALF = MF_COLS / 2;
  for (int e = threadIdx.x; e < ROWS * HALF; e += MF_NT) {
    const int row = e / HALF, cp = e - row * HALF;
    const int gy = r0 + row, gx = q0 + 2 * cp;
    float v0 = 0.f, v1 = 0.f;
    if (gy >= 0 && gy < H) {
      const float* rp = src + (int64_t)gy * W;
      if (gx >= 0 && gx < W) v0 = rp[gx];
      if (gx + 1 >= 0 && gx + 1 < W) v1 = rp[gx + 1];
    }
    unsigned short h0, l0, h1, l1;
    split_bf16(v0, h0, l0);
    split_bf16(v1, h1, l1);
    const int o = row * MF_PITCH + 2 * cp;
    *reinterpret_cast<unsigned int*>(sh_hi + o) = (unsigned int)h0 | ((unsigned int)h1 << 16);
    *reinterpret_cast<unsigned int*>(sh_lo + o) = (unsigned int)l0 | ((unsigned int)l1 << 16);
  }
}

// One class of kernel rows a = r + 16 m, m < NM: accumulate into acc.
template <int NM, int NS>
__device__ inline void mfma_class(int r, const unsigned short* sh_hi, const unsigned short* sh_lo,
                                  const bf16x8* __restrict__ tab_t, int row_base, int col_base,
                                  f32x4 (&acc)[MF_BR][MF_BC]) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  // Toeplitz fragments U_a for a = r + 16m, both k-halves, hi (and lo)
  bf16x8 T[NM][2][2];
#pragma unroll
  for (int m = 0; m < NM; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int s = 0; s < (NS == 3 ? 2 : 1); ++s)
        T[m][h][s] = tab_t[(((r + 16 * m) * 2 + h) * 2 + s) * 64 + lane];
#pragma unroll
  for (int rho = 0; rho < MF_BR + NM - 1; ++rho) {
    const int lrow = row_base + r + 16 * rho + i;
#pragma unroll
    for (int kap = 0; kap < MF_BC + 2; ++kap) {
      const int o = lrow * MF_PITCH + col_base + 16 * kap + 8 * g;
      const bf16x8 Ah = *reinterpret_cast<const bf16x8*>(sh_hi + o);
      bf16x8 Al;
      if (NS == 3) Al = *reinterpret_cast<const bf16x8*>(sh_lo + o);
#pragma unroll
      for (int m = 0; m < NM; ++m) {
        const int beta = rho - m;
        if (beta < 0 || beta >= MF_BR) continue;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int gam = kap - 2 * h;
          if (gam < 0 || gam >= MF_BC) continue;
          acc[beta][gam] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, T[m][h][0], acc[beta][gam], 0, 0, 0);
          if (NS == 3) {
            acc[beta][gam] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, T[m][h][0], acc[beta][gam], 0, 0, 0);
            acc[beta][gam] =
                __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, T[m][h][1], acc[beta][gam], 0, 0, 0);
          }
        }
      }
    }
  }
}

// All kernel rows of one frame.
template <int KT, int NS>
__device__ inline void mfma_frame(const unsigned short* sh_hi, const unsigned short* sh_lo,
                                  const bf16x8* __restrict__ tab_t, int row_base, int col_base,
                                  f32x4 (&acc)[MF_BR][MF_BC]) {
  // classes r with 3, 2 and 1 members (KT = 43: r<=10 -> 3, else 2; KT = 15: r<=14 -> 1)
  constexpr int R3 = KT > 32 ? KT - 32 : 0;
  constexpr int R2 = KT > 16 ? (KT - 16 < 16 ? KT - 16 : 16) : 0;
  constexpr int R1 = KT < 16 ? KT : 16;
  int r = 0;
  for (; r < R3; ++r) mfma_class<3, NS>(r, sh_hi, sh_lo, tab_t, row_base, col_base, acc);
  for (; r < R2; ++r) mfma_class<2, NS>(r, sh_hi, sh_lo, tab_t, row_base, col_base, acc);
  for (; r < R1; ++r) mfma_class<1, NS>(r, sh_hi, sh_lo, tab_t, row_base, col_base, acc);
}

// Forward: r_t = u_t * (f_t * x) for the frames of this group, x tile staged once.
template <int KT, int NS>
__global__ __launch_bounds__(MF_NT) void mfma_fwd_kernel(MfmaLaunch a) {
  constexpr int c = (KT - 1) / 2;
  constexpr int ROWS = MF_TH + KT - 1;
  __shared__ __align__(16) unsigned short sh_hi[ROWS * MF_PITCH];
  __shared__ __align__(16) unsigned short sh_lo[ROWS * MF_PITCH];
  __shared__ double red[MF_NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int tiles_x = (a.W + MF_TW - 1) / MF_TW;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int k0 = ty * MF_TH, l0 = tx * MF_TW;
  stage_tile<ROWS>(a.in, a.H, a.W, k0 - c, l0 - c, sh_hi, sh_lo);
  __syncthreads();

  const int t0 = blockIdx.y * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const int64_t N = (int64_t)a.H * a.W;
  double llp = 0.0;
  for (int t = t0; t < t1; ++t) {
    f32x4 acc[MF_BR][MF_BC];
#pragma unroll
    for (int b = 0; b < MF_BR; ++b)
#pragma unroll
      for (int q = 0; q < MF_BC; ++q) acc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8* tab_t = reinterpret_cast<const bf16x8*>(a.tab) + (int64_t)t * KT * 4 * 64;
    mfma_frame<KT, NS>(sh_hi, sh_lo, tab_t, wr * 64, wc * 64, acc);
    const int64_t base = (int64_t)t * N;
#pragma unroll
    for (int b = 0; b < MF_BR; ++b)
#pragma unroll
      for (int q = 0; q < MF_BC; ++q) {
        const int l = l0 + wc * 64 + 16 * q + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = k0 + wr * 64 + 16 * b + 4 * (lane >> 4) + v;
          if (k < a.H && l < a.W) {
            const int64_t idx = base + (int64_t)k * a.W + l;
            const float m = acc[b][q][v];
            if (a.u == nullptr) {
              a.out[idx] = m;
            } else {
              const float uu = a.u[idx];
              if (a.out) a.out[idx] = uu * m;
              if (a.part != nullptr && uu > 0.f) {
                const double d = (double)a.y[idx] - (double)m;
                llp += (double)uu * d * d;
              }
            }
          }
        }
      }
  }
  if (a.part != nullptr) {
    const double s = block_sum<MF_NT>(llp, red);
    if (threadIdx.x == 0) a.part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
  }
}

__device__ inline float mf_update_value(float xo, float Bv, float Dn) {
  if (xo == 0.f) return 0.f;
  if (Dn == 0.f) return xo;
  const float q = fmaxf(Bv, 0.f) / Dn;
  return xo * q;
}

// Adjoint: sum over the frames of this group of F_t^T r_t; the r_t tile is
// staged per frame.  Epilogue: partial plane, or the fused update of Eq. (2).
template <int KT, int NS>
__global__ __launch_bounds__(MF_NT) void mfma_adj_kernel(MfmaLaunch a) {
  constexpr int c = (KT - 1) / 2;
  constexpr int ROWS = MF_TH + KT - 1;
  __shared__ __align__(16) unsigned short sh_hi[ROWS * MF_PITCH];
  __shared__ __align__(16) unsigned short sh_lo[ROWS * MF_PITCH];
  __shared__ double red[2 * MF_NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int tiles_x = (a.W + MF_TW - 1) / MF_TW;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int k0 = ty * MF_TH, l0 = tx * MF_TW;
  const int64_t N = (int64_t)a.H * a.W;

  f32x4 acc[MF_BR][MF_BC];
#pragma unroll
  for (int b = 0; b < MF_BR; ++b)
#pragma unroll
    for (int q = 0; q < MF_BC; ++q) acc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int t0 = blockIdx.y * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();
    stage_tile<ROWS>(a.in + (int64_t)t * N, a.H, a.W, k0 - c, l0 - c, sh_hi, sh_lo);
    __syncthreads();
    const bf16x8* tab_t = reinterpret_cast<const bf16x8*>(a.tab) + (int64_t)t * KT * 4 * 64;
    mfma_frame<KT, NS>(sh_hi, sh_lo, tab_t, wr * 64, wc * 64, acc);
  }

  double dsq = 0.0, xsq = 0.0;
#pragma unroll
  for (int b = 0; b < MF_BR; ++b)
#pragma unroll
    for (int q = 0; q < MF_BC; ++q) {
      const int l = l0 + wc * 64 + 16 * q + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = k0 + wr * 64 + 16 * b + 4 * (lane >> 4) + v;
        if (k < a.H && l < a.W) {
          const int64_t idx = (int64_t)k * a.W + l;
          if (a.fused) {
            const float xo = a.x[idx];
            const float xn = mf_update_value(xo, a.B[idx], acc[b][q][v]);
            a.x[idx] = xn;
            const double d = (double)xn - (double)xo;
            dsq += d * d;
            xsq += (double)xo * (double)xo;
          } else {
            a.plane[(int64_t)blockIdx.y * N + idx] = acc[b][q][v];
          }
        }
      }
    }
  if (a.fused && a.part != nullptr) {
    const double s1 = block_sum<MF_NT>(dsq, red);
    __syncthreads();
    const double s2 = block_sum<MF_NT>(xsq, red + MF_NT / 64);
    if (threadIdx.x == 0) {
      a.part[2 * blockIdx.x] = s1;
      a.part[2 * blockIdx.x + 1] = s2;
    }
  }
}

// Toeplitz fragment tables, one block per (frame, kernel row a): entry
// [t][a][h][s][lane] holds the 8 bf16 values U_a[32h + 8(lane/16) + e][lane%16],
// e = 0..7, of part s (0 = hi, 1 = lo) of g = flip(f) (dir 0, forward) or
// g = f (dir 1, adjoint), f zero-padded from K to KT.
__global__ __launch_bounds__(256) void mfma_table_kernel(const float* psf, int K, int KT, int dir,
                                                         unsigned short* tab) {
  const int t = blockIdx.x, a = blockIdx.y;
  const int off = (KT - K) / 2;
  const float* f = psf + (int64_t)t * K * K;
  const int idx = threadIdx.x;          // (h, s, lane) = 2 x 2 x 64
  const int lane = idx & 63, s = (idx >> 6) & 1, h = idx >> 7;
  const int j = lane & 15, gq = lane >> 4;
  unsigned short* dst = tab + ((((int64_t)t * KT + a) * 2 + h) * 2 + s) * 64 * 8 + lane * 8;
  for (int e = 0; e < 8; ++e) {
    const int p = 32 * h + 8 * gq + e;
    const int b = p - j;                 // column of g
    float gv = 0.f;
    if (b >= 0 && b < KT) {
      // g[a][b]: forward uses the 180-degree flip of f
      const int fa = dir == 0 ? KT - 1 - a : a;
      const int fb = dir == 0 ? KT - 1 - b : b;
      const int ia = fa - off, ib = fb - off;
      if (ia >= 0 && ia < K && ib >= 0 && ib < K) gv = f[ia * K + ib];
    }
    unsigned short hi, lo;
    split_bf16(gv, hi, lo);
    dst[e] = s == 0 ? hi : lo;
  }
}

hipError_t launch_mfma_tables(const Geometry& g, const float* psf, void* tab_fwd, void* tab_adj,
                              hipStream_t s) {
  dim3 grid(g.n, g.KT);
  hipLaunchKernelGGL(mfma_table_kernel, grid, dim3(256), 0, s, psf, g.K, g.KT, 0,
                     static_cast<unsigned short*>(tab_fwd));
  hipLaunchKernelGGL(mfma_table_kernel, grid, dim3(256), 0, s, psf, g.K, g.KT, 1,
                     static_cast<unsigned short*>(tab_adj));
  return hipGetLastError();
}

int mfma_tile_h() { return MF_TH; }
int mfma_tile_w() { return MF_TW; }

hipError_t launch_mfma(const Geometry& g, int dir, int tiles, int groups, const MfmaLaunch& a,
                       hipStream_t s) {
  dim3 grid(tiles, groups), block(MF_NT);
  const bool split = g.precision == EM_BF16_SPLIT;
  if (dir == 0) {
    if (g.KT == KT_LARGE) {
      if (split) hipLaunchKernelGGL((mfma_fwd_kernel<KT_LARGE, 3>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mfma_fwd_kernel<KT_LARGE, 1>), grid, block, 0, s, a);
    } else {
      if (split) hipLaunchKernelGGL((mfma_fwd_kernel<KT_SMALL, 3>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mfma_fwd_kernel<KT_SMALL, 1>), grid, block, 0, s, a);
    }
  } else {
    if (g.KT == KT_LARGE) {
      if (split) hipLaunchKernelGGL((mfma_adj_kernel<KT_LARGE, 3>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mfma_adj_kernel<KT_LARGE, 1>), grid, block, 0, s, a);
    } else {
      if (split) hipLaunchKernelGGL((mfma_adj_kernel<KT_SMALL, 3>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((mfma_adj_kernel<KT_SMALL, 1>), grid, block, 0, s, a);
    }
  }
  return hipGetLastError();
}

}  // namespace em
