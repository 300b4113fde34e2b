// em_mfma2n.hip -- forward convolution of the super-resolution iteration
// (arXiv:2302.05804, Sec. 2, Eq. (3) inside Eq. (2)) on the matrix cores with
// the frames in the N dimension of the products: FP16 split and BF16 split
// forms, jobs of at least M2N_MIN_FRAMES frames.
//
// With g_t the flipped 44 x 44 box-extended kernel of frame t (as in
// em_mfma2.hip),
//   m_t[I][J] = sum_{a,b < 44} g_t[a][b] x[2I - 21 + a][2J - 21 + b].
// The image operand x is the same for every frame, so one
// v_mfma_f32_16x16x32_f16 takes 16 output pixels of one row (M), 32 taps of one
// kernel row (K) and 16 frames (N):
//   A[i][k] = x[R][2(J0 + i) - 21 + b0 + k],   B[k][j] = g_{t0 + j}[a][b0 + k],
// R = 2I - 21 + a, and no Toeplitz zeros enter the products (the column
// Toeplitz operand of the other sr = 2 forward is 44/96 dense).  The 44 taps of
// a kernel row are one 32-tap chunk and a 16-tap tail (taps 32..47, 44..47
// zero); the tails of kernel rows 2p and 2p + 1 share one chunk (k < 16 from
// latent row R, k >= 16 from R + 1), so a row pair p = 0..21 takes three chunks.
//
// Output row I reads latent rows 2I - 21 + 2p (+1) for pair p: the A fragments
// of pair p of output row I are those of pair p - 1 of output row I + 1.  A wave
// owning BR consecutive output rows keeps a window of BR + 1 latent row pairs in
// registers and reads one new pair from LDS per step (each A fragment serves BR
// output rows).  The B fragments of a pair (hi and lo parts of the three chunks,
// one binary16 scale per frame) come from a per-group table in global memory,
// which stays in L2, and each serves BR x BC products.
// FP16 split: the staged x tile is binary16 with a power-of-two scale, the PSF
// parts carry one per frame, and the epilogue removes both scales exactly; the
// PSF's lo part enters on kernel rows 11..32 only, as in the other FP16 split
// sr = 2 forward.  BF16 split: the staged tile holds the hi and lo bf16 planes
// of x, and every kernel row takes x_hi g_hi + x_lo g_hi + x_hi g_lo, as the
// sr = 2 adjoint of that form does; the two image planes double the register
// window, so its workgroups cover 16 x 32 frame pixels.
#include "em_device.h"
#include "em_internal.h"
#include "em_mfma_common.h"

#include <type_traits>

namespace em {

namespace {

constexpr int M2N_PAIRS = 22;                    // kernel row pairs (44 rows)
constexpr int M2N_NF = 6;                        // B fragments per pair
constexpr int64_t M2N_GROUP_FRAGS = (int64_t)M2N_PAIRS * M2N_NF * 64;   // 16-byte fragments
constexpr size_t M2N_GROUP_BYTES = (size_t)M2N_GROUP_FRAGS * 16;

// kernel rows of the 44 x 44 box-extended kernel that take the PSF's lo part
template <int PREC>
__host__ __device__ constexpr bool m2n_lo_row(int a) {
  return PREC != EM_FP16_SPLIT || (a >= 11 && a <= 32);
}

// LDS row pitch (halves): at least `cols`, even, and half of it (the distance
// in dwords between consecutive latent rows) 20..44 mod 64, so that the two
// rows read by one tail-chunk fragment fall on different banks.
__host__ __device__ constexpr int m2n_pitch(int cols) {
  int p = cols + (cols & 1);
  while ((p / 2) % 64 < 20 || (p / 2) % 64 > 44) p += 2;
  return p;
}

// BR output rows x BC blocks of 16 output columns per wave, WR x WC waves.
template <int BR_, int BC_, int WR_, int WC_, int PREC_ = EM_FP16_SPLIT>
struct M2N {
  static constexpr int BR = BR_, BC = BC_, WR = WR_, WC = WC_, PREC = PREC_;
  using P = Prec<PREC_>;
  using frag = typename P::frag;
  static constexpr int NA = P::NA;                  // image planes
  static constexpr bool R16 = PREC_ == EM_FP16_SPLIT;   // may write binary16 r planes
  static constexpr int NW = WR * WC, NT = 64 * NW;
  static constexpr int TH = BR * WR, TW = 16 * BC * WC;   // frame pixels per workgroup
  static constexpr int ROWS = 2 * TH + 42;                 // latent rows staged
  static constexpr int COLS = 2 * TW + 46;                 // latent columns staged
  static constexpr int PITCH = m2n_pitch(COLS);
  // binary16 r planes: the workgroup's outputs of all 16 frames go through an LDS
  // staging tile so that most stores are 16-byte runs.  A plane holds output
  // column J at plane column J + 11, so the runs that start on 16-byte
  // boundaries begin at output columns J0 + LEAD + 8 j.
  static constexpr int LEAD = (8 - 11 % 8) % 8;
  static constexpr int S0 = (8 - LEAD) % 8;        // staging column of output column J0
  static constexpr int NRUN = (TW - LEAD) / 8;
  static constexpr int TAIL = TW - LEAD - 8 * NRUN;
  static constexpr int SP = (S0 + TW + 7) / 8 * 8;  // staging row pitch (halves)
  static constexpr int FS = TH * SP + 8;            // staging frame stride (halves)
};

// Eight 16-bit values of one latent row of a staged plane, starting at an
// even column (dword reads: the start is 4-byte aligned only).
template <class F>
__device__ inline F m2n_ld8(const unsigned short* __restrict__ sh, int off) {
  const uint32_t* p = reinterpret_cast<const uint32_t*>(sh + off);
  uint4 v;
  v.x = p[0];
  v.y = p[1];
  v.z = p[2];
  v.w = p[3];
  return __builtin_bit_cast(F, v);
}

template <class F>
__device__ inline F m2n_ldB(const F* __restrict__ tab, int p, int f) {
  return tab[(p * M2N_NF + f) * 64];
}

template <class C, bool ROB>
__device__ inline void m2n_body(const MfmaLaunch& a, const int tile, const int group) {
  using F = typename C::frag;
  constexpr bool STG = !ROB && C::R16;   // binary16 r planes possible
  __shared__ __align__(16) unsigned short sh[C::NA][C::ROWS * C::PITCH];
  __shared__ double red[C::NW];
  __shared__ float redf[C::NW];
  __shared__ __align__(16) std::conditional_t<STG, unsigned short[M2N_FPG * C::FS],
                                              unsigned short[8]> stg;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w / C::WC, wc = w % C::WC;
  const int tiles_x = (a.W + C::TW - 1) / C::TW;     // a.H, a.W: frame grid
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int I0 = ty * C::TH, J0 = tx * C::TW;
  const int t0 = group * M2N_FPG;
  const int sx = stage_tile<C::PREC, C::ROWS, C::COLS, C::PITCH, C::NT>(
      a.in, 2 * a.H, 2 * a.W, 2 * I0 - 21, 2 * J0 - 21, sh, redf);
  __syncthreads();

  const int i = lane & 15, gq = lane >> 4;
  const unsigned short* base = &sh[0][0];
  constexpr int PLANE = C::ROWS * C::PITCH;
  // tile row of latent row 2 (I0 + wr BR) - 21 (pair 0 of the wave's row 0) and
  // tile column of this lane's output column in block 0, times 2
  const int row0 = 2 * wr * C::BR;
  const int col0 = 2 * (wc * 16 * C::BC + i);
  // A fragments of latent row pair q: full chunk of row 2q, of row 2q + 1, tail
  const int off_f0 = row0 * C::PITCH + col0 + 8 * gq;
  const int off_f1 = off_f0 + C::PITCH;
  const int off_t = (row0 + (gq >> 1)) * C::PITCH + col0 + 32 + 8 * (gq & 1);
  const F* tab = reinterpret_cast<const F*>(a.tab) + (int64_t)group * M2N_GROUP_FRAGS + lane;

  constexpr int NS = C::BR + 1;   // window slots
  F F0[NS][C::BC][C::NA], F1[NS][C::BC][C::NA], FT[NS][C::BC][C::NA];
  f32x4 acc[C::BR][C::BC];
#pragma unroll
  for (int b = 0; b < C::BR; ++b)
#pragma unroll
    for (int c = 0; c < C::BC; ++c) acc[b][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < C::BR; ++q)
#pragma unroll
    for (int c = 0; c < C::BC; ++c)
#pragma unroll
      for (int pa = 0; pa < C::NA; ++pa) {
        F0[q][c][pa] = m2n_ld8<F>(base + pa * PLANE, off_f0 + 2 * q * C::PITCH + 32 * c);
        F1[q][c][pa] = m2n_ld8<F>(base + pa * PLANE, off_f1 + 2 * q * C::PITCH + 32 * c);
        FT[q][c][pa] = m2n_ld8<F>(base + pa * PLANE, off_t + 2 * q * C::PITCH + 32 * c);
      }
  F G[M2N_NF], Gn[M2N_NF];
#pragma unroll
  for (int f = 0; f < M2N_NF; ++f) G[f] = m2n_ldB<F>(tab, 0, f);

#pragma unroll
  for (int p = 0; p < M2N_PAIRS; ++p) {
    const bool lo0 = m2n_lo_row<C::PREC>(2 * p), lo1 = m2n_lo_row<C::PREC>(2 * p + 1);
    if (p + 1 < M2N_PAIRS) {
      // the window's next pair (used from step p + 1 on) and the next B fragments
      const int q = p + C::BR, s = q % NS;
#pragma unroll
      for (int c = 0; c < C::BC; ++c)
#pragma unroll
        for (int pa = 0; pa < C::NA; ++pa) {
          F0[s][c][pa] = m2n_ld8<F>(base + pa * PLANE, off_f0 + 2 * q * C::PITCH + 32 * c);
          F1[s][c][pa] = m2n_ld8<F>(base + pa * PLANE, off_f1 + 2 * q * C::PITCH + 32 * c);
          FT[s][c][pa] = m2n_ld8<F>(base + pa * PLANE, off_t + 2 * q * C::PITCH + 32 * c);
        }
      const bool nlo0 = m2n_lo_row<C::PREC>(2 * p + 2), nlo1 = m2n_lo_row<C::PREC>(2 * p + 3);
#pragma unroll
      for (int f = 0; f < M2N_NF; ++f) {
        const bool need = (f & 1) == 0 || (f == 1 && nlo0) || (f == 3 && nlo1) ||
                          (f == 5 && (nlo0 || nlo1));
        if (need) Gn[f] = m2n_ldB<F>(tab, p + 1, f);
      }
    }
    // keep these loads ahead of this step's products (the scheduler would
    // otherwise sink them next to their first use, exposing their latency)
    __builtin_amdgcn_sched_barrier(0);
    // products of pair p; consecutive products write different accumulators.
    // kind % 3 is the chunk (row 2p, row 2p + 1, tail); FP16 split: kinds 0-2
    // x g_hi, 3-5 x g_lo; BF16 split: 0-2 x_hi g_hi, 3-5 x_lo g_hi, 6-8 x_hi g_lo
    constexpr int NKIND = C::NA == 2 ? 9 : 6;
#pragma unroll
    for (int kind = 0; kind < NKIND; ++kind) {
      const int ch = kind % 3;
      const bool glo = kind >= (C::NA == 2 ? 6 : 3);
      const int pa = (C::NA == 2 && kind >= 3 && kind < 6) ? 1 : 0;
      if (glo && ch == 0 && !lo0) continue;
      if (glo && ch == 1 && !lo1) continue;
      if (glo && ch == 2 && !(lo0 || lo1)) continue;
      const int f = 2 * ch + (glo ? 1 : 0);
#pragma unroll
      for (int b = 0; b < C::BR; ++b) {
        const int s = (b + p) % NS;
#pragma unroll
        for (int c = 0; c < C::BC; ++c) {
          const F& A = ch == 0 ? F0[s][c][pa] : (ch == 1 ? F1[s][c][pa] : FT[s][c][pa]);
          acc[b][c] = C::P::mma(A, G[f], acc[b][c]);
        }
      }
    }
    if (p + 1 < M2N_PAIRS) {
#pragma unroll
      for (int f = 0; f < M2N_NF; ++f) G[f] = Gn[f];
    }
  }

  // epilogue: lane (j + 16 gq) holds frame t0 + j at columns 4 gq .. 4 gq + 3 of
  // each 16-column block
  const int t = t0 + (lane & 15);
  const bool tv = t < a.n;
  const int tc = tv ? t : a.n - 1;
  const int* ex = reinterpret_cast<const int*>(static_cast<const char*>(a.tab) +
                                               (size_t)((a.n + M2N_FPG - 1) / M2N_FPG) *
                                                   M2N_GROUP_BYTES);
  const int unscale = -(sx + ex[tc]);
  const int64_t N = (int64_t)a.H * a.W;
  // u == nullptr: the raw m (operator form); out == nullptr: partials only
  const float* ut = a.u ? a.u + (int64_t)tc * N : nullptr;
  const float* yt = a.y ? a.y + (int64_t)tc * N : nullptr;
  float* ot = a.out ? a.out + (int64_t)tc * N : nullptr;
  float* oyt = ROB ? a.out_y + (int64_t)tc * N : nullptr;
  // binary16 r planes (the Gaussian iteration): 2^e16[t] u m at plane pixel
  // (I + 11, J + 11) instead of r, through the staging tile
  const bool to16 = STG && a.r16 != nullptr;     // uniform over the workgroup
  const int e16 = to16 ? a.e16[tc] : 0;
  const bool want_ll = a.part != nullptr;
  const float nu = a.nu, nu1 = a.nu + 1.f;
  // four consecutive pixels per lane and block: 16-byte accesses when rows and
  // bases allow (frame width a multiple of 4, 16-byte aligned planes)
  const bool al =
      (a.W & 3) == 0 &&
      ((reinterpret_cast<uintptr_t>(ut) | reinterpret_cast<uintptr_t>(yt) |
        reinterpret_cast<uintptr_t>(ot) | reinterpret_cast<uintptr_t>(oyt)) & 15) == 0;
  double llp = 0.0;
#pragma unroll
  for (int b = 0; b < C::BR; ++b) {
    const int I = I0 + wr * C::BR + b;
#pragma unroll
    for (int c = 0; c < C::BC; ++c) {
      const int Jb = J0 + 16 * (wc * C::BC + c) + 4 * gq;
      const bool vec = al && Jb + 3 < a.W;
      float uu[4], yy[4];
      const int Ic = min(I, a.H - 1);
      if (vec) {
        const int64_t o = (int64_t)Ic * a.W + Jb;
        const float4 u4 = ut ? *reinterpret_cast<const float4*>(ut + o) : make_float4(1.f, 1.f, 1.f, 1.f);
        const float4 y4 = (ROB || want_ll) ? *reinterpret_cast<const float4*>(yt + o)
                                           : make_float4(0.f, 0.f, 0.f, 0.f);
        uu[0] = u4.x; uu[1] = u4.y; uu[2] = u4.z; uu[3] = u4.w;
        yy[0] = y4.x; yy[1] = y4.y; yy[2] = y4.z; yy[3] = y4.w;
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t o = (int64_t)Ic * a.W + min(Jb + v, a.W - 1);
          uu[v] = ut ? ut[o] : 1.f;
          yy[v] = (ROB || want_ll) ? yt[o] : 0.f;
        }
      }
      if (!tv || I >= a.H) continue;
      float ro[4], ryo[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float m = ldexpf(acc[b][c][v], unscale);
        const float u = uu[v];
        const bool in = Jb + v < a.W;
        if constexpr (ROB) {
          ro[v] = 0.f;
          ryo[v] = 0.f;
          if (u > 0.f) {
            const float y = yy[v];
            const float d = y - m;
            const float wgt = nu1 / (nu + u * d * d);
            ro[v] = (u * wgt) * m;
            ryo[v] = (u * wgt) * y;
            if (want_ll && in) {
              const double dd = (double)y - (double)m;
              llp += ((double)nu + 1.0) * log1p((double)u * dd * dd / (double)nu) - a.lcst;
            }
          }
        } else {
          ro[v] = ut ? u * m : m;
          ryo[v] = 0.f;
          if (want_ll && in && u > 0.f) {
            const double d = (double)yy[v] - (double)m;
            llp += (double)u * d * d;
          }
        }
      }
      const int64_t o = (int64_t)I * a.W + Jb;
      if constexpr (STG) {
        if (to16) {
          unsigned short* srow =
              &stg[(lane & 15) * C::FS + (I - I0) * C::SP + C::S0 + (Jb - J0)];
#pragma unroll
          for (int v = 0; v < 4; ++v) srow[v] = f16_bits((_Float16)ldexpf(ro[v], e16));
          continue;
        }
      }
      if (vec) {
        if (ot) *reinterpret_cast<float4*>(ot + o) = make_float4(ro[0], ro[1], ro[2], ro[3]);
        if constexpr (ROB)
          *reinterpret_cast<float4*>(oyt + o) = make_float4(ryo[0], ryo[1], ryo[2], ryo[3]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (Jb + v >= a.W) continue;
          if (ot) ot[o + v] = ro[v];
          if constexpr (ROB) oyt[o + v] = ryo[v];
        }
      }
    }
  }
  if constexpr (STG) {
    if (to16) {
      __syncthreads();
      constexpr int SLOTS = C::NRUN + 1;   // per frame row: the runs, then lead and tail
      for (int e = threadIdx.x; e < M2N_FPG * C::TH * SLOTS; e += C::NT) {
        const int f = e / (C::TH * SLOTS), rem = e - f * (C::TH * SLOTS);
        const int rr = rem / SLOTS, j = rem - rr * SLOTS;
        const int tf = t0 + f, I = I0 + rr;
        if (tf >= a.n || I >= a.H) continue;
        unsigned short* prow = a.r16 + (int64_t)tf * a.s16 + (int64_t)(I + 11) * a.p16 + 11;
        const unsigned short* srow = &stg[f * C::FS + rr * C::SP + C::S0];
        if (j < C::NRUN) {
          const int lc = J0 + C::LEAD + 8 * j;
          if (lc + 7 < a.W) {
            *reinterpret_cast<uint4*>(prow + lc) =
                *reinterpret_cast<const uint4*>(srow + C::LEAD + 8 * j);
          } else {
#pragma unroll
            for (int i = 0; i < 8; ++i)
              if (lc + i < a.W) prow[lc + i] = srow[C::LEAD + 8 * j + i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < C::LEAD; ++i)
            if (J0 + i < a.W) prow[J0 + i] = srow[i];
#pragma unroll
          for (int i = 0; i < C::TAIL; ++i) {
            const int lc = J0 + C::LEAD + 8 * C::NRUN + i;
            if (lc < a.W) prow[lc] = srow[C::LEAD + 8 * C::NRUN + i];
          }
        }
      }
    }
  }
  if (want_ll) {
    const double s = block_sum<C::NT>(llp, red);
    if (threadIdx.x == 0) a.part[(int64_t)group * a.ntiles + tile] = s;
  }
}

template <class C>
__global__ __launch_bounds__(C::NT) void m2n_kernel(MfmaLaunch a) {
  m2n_body<C, false>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2n_t_kernel(MfmaLaunch a) {
  m2n_body<C, true>(a, blockIdx.x, blockIdx.y);
}
// serving: work items (descriptor, tile, group) of every job of the round
template <class C, bool ROB>
__global__ __launch_bounds__(C::NT) void m2n_batched(const MfmaLaunch* __restrict__ descs,
                                                     const int4* __restrict__ items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    m2n_body<C, ROB>(descs[w.x], w.y, w.z);
    __syncthreads();
  }
}

// Table of one frame group (one block per group and pair): fragment
// [group][p][f][lane], f = 2 ch + s for chunk ch (0: taps 0..31 of row 2p,
// 1: of row 2p + 1, 2: taps 32..47 of rows 2p (k < 16) and 2p + 1 (k >= 16)) and
// part s (0 hi, 1 lo; FP16 split: lo is zero on rows outside 11..32); lane
// j + 16 gq holds B[8 gq + e][j] of frame 16 group + j (zero beyond n).  After
// all groups: the n frames' scale exponents (FP16 split: f16_scale_exp of the
// largest |k_t|; BF16 split: 0, no scale).
template <int PREC>
__global__ __launch_bounds__(384) void m2n_table_kernel(const float* psf, int n, int K,
                                                       unsigned short* tab) {
  __shared__ int sexp[M2N_FPG];
  const int grp = blockIdx.x, p = blockIdx.y;
  const int off = (43 - K) / 2;
  auto kk = [&](int t, int a, int b) -> float {   // 44 x 44 box-extended kernel of frame t
    const float* f = psf + (int64_t)t * K * K;
    auto fp = [&](int r, int q) -> float {
      const int ia = r - off, ib = q - off;
      if (ia < 0 || ia >= K || ib < 0 || ib >= K) return 0.f;
      return f[ia * K + ib];
    };
    if (a < 0 || a >= 44 || b < 0 || b >= 44) return 0.f;
    return (fp(a - 1, b - 1) + fp(a - 1, b)) + (fp(a, b - 1) + fp(a, b));
  };
  // per-frame scale exponents: one wave per frame of the group
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = w; j < M2N_FPG; j += 6) {
    const int t = grp * M2N_FPG + j;
    float mx = 0.f;
    if (t < n)
      for (int e = lane; e < 44 * 44; e += 64) mx = fmaxf(mx, fabsf(kk(t, e / 44, e % 44)));
    mx = wave_max(mx);
    if (lane == 0) {
      sexp[j] = PREC == EM_FP16_SPLIT ? f16_scale_exp(mx) : 0;
      if (t < n && p == 0)
        reinterpret_cast<int*>(reinterpret_cast<char*>(tab) +
                               (size_t)((n + M2N_FPG - 1) / M2N_FPG) * M2N_GROUP_BYTES)[t] =
            sexp[j];
    }
  }
  __syncthreads();
  // idx = (f, lane): 6 x 64
  const int f = threadIdx.x >> 6, s = f & 1, ch = f >> 1;
  const int j = lane & 15, gq = lane >> 4, t = grp * M2N_FPG + j;
  unsigned short* dst =
      tab + (((int64_t)grp * M2N_PAIRS + p) * M2N_NF + f) * 64 * 8 + lane * 8;
  for (int e = 0; e < 8; ++e) {
    const int k = 8 * gq + e;
    int a, b;
    if (ch < 2) {
      a = 2 * p + ch;
      b = k;
    } else {
      a = 2 * p + (k >= 16 ? 1 : 0);
      b = 32 + (k & 15);
    }
    float gv = 0.f;
    if (t < n && b < 44) gv = kk(t, 43 - a, 43 - b);
    unsigned short v = table_part<PREC>(ldexpf(gv, sexp[j]), s);
    if (s == 1 && !m2n_lo_row<PREC>(a)) v = 0;
    dst[e] = v;
  }
}

// FP16 split variants: 0: 8 waves (2 x 4) of 8 rows x 1 block; 1: 8 waves
// (4 x 2) of 4 rows x 2 blocks; 2: 8 waves (8 x 1) of 2 rows x 4 blocks, each
// covering 16 x 64 frame pixels.  BF16 split (two image planes in the window):
// 0 and 2: 8 waves (4 x 2) of 4 rows x 1 block; 1: 8 waves (8 x 1) of 2 rows x
// 2 blocks, each covering 16 x 32 frame pixels (a third shape within the
// register budget of 8-wave workgroups would leave one output row per wave).
using N0 = M2N<8, 1, 2, 4>;
using N1 = M2N<4, 2, 4, 2>;
using N2 = M2N<2, 4, 8, 1>;
using NB0 = M2N<4, 1, 4, 2, EM_BF16_SPLIT>;
using NB1 = M2N<2, 2, 8, 1, EM_BF16_SPLIT>;
template <class C>
constexpr bool m2n_tile_ok() {
  return C::TH == M2N_TH && C::TW == m2n_tile_w(C::PREC);
}
static_assert(m2n_tile_ok<N0>() && m2n_tile_ok<N1>() && m2n_tile_ok<N2>() &&
                  m2n_tile_ok<NB0>() && m2n_tile_ok<NB1>(),
              "tile");

}  // namespace

size_t mfma2n_table_bytes(int n) {
  return (size_t)((n + M2N_FPG - 1) / M2N_FPG) * M2N_GROUP_BYTES + (size_t)n * sizeof(int);
}

hipError_t launch_mfma2n_table(const Geometry& g, const float* psf, void* tab, hipStream_t s) {
  const dim3 grid((g.n + M2N_FPG - 1) / M2N_FPG, M2N_PAIRS);
  if (g.precision == EM_FP16_SPLIT)
    hipLaunchKernelGGL(m2n_table_kernel<EM_FP16_SPLIT>, grid, dim3(384), 0, s, psf, g.n, g.K,
                       static_cast<unsigned short*>(tab));
  else if (g.precision == EM_BF16_SPLIT)
    hipLaunchKernelGGL(m2n_table_kernel<EM_BF16_SPLIT>, grid, dim3(384), 0, s, psf, g.n, g.K,
                       static_cast<unsigned short*>(tab));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

bool mfma2n_desc_ok(const Geometry& g, int tiles, int groups, const MfmaLaunch& a) {
  return uses_m2n(g) && a.H == g.Hf && a.W == g.Wf && a.fpg == M2N_FPG &&
         (a.r16 == nullptr || (a.out == nullptr && a.out_y == nullptr)) &&
         launch_grid_ok(tiles, groups, a.ntiles, a.n, a.fpg, a.H, a.W, M2N_TH,
                        m2n_tile_w(g.precision));
}

hipError_t launch_mfma2n(const Geometry& g, int variant, int tiles, int groups,
                         const MfmaLaunch& a, hipStream_t s) {
  if (!mfma2n_desc_ok(g, tiles, groups, a)) return hipErrorInvalidValue;
  const dim3 grid(tiles, groups);
  const bool rob = a.out_y != nullptr;
  if (g.precision == EM_BF16_SPLIT) {
    if (variant == 1) {
      if (rob) hipLaunchKernelGGL(m2n_t_kernel<NB1>, grid, dim3(NB1::NT), 0, s, a);
      else hipLaunchKernelGGL(m2n_kernel<NB1>, grid, dim3(NB1::NT), 0, s, a);
    } else {
      if (rob) hipLaunchKernelGGL(m2n_t_kernel<NB0>, grid, dim3(NB0::NT), 0, s, a);
      else hipLaunchKernelGGL(m2n_kernel<NB0>, grid, dim3(NB0::NT), 0, s, a);
    }
    return hipGetLastError();
  }
  if (variant == 1) {
    if (rob) hipLaunchKernelGGL(m2n_t_kernel<N1>, grid, dim3(N1::NT), 0, s, a);
    else hipLaunchKernelGGL(m2n_kernel<N1>, grid, dim3(N1::NT), 0, s, a);
  } else if (variant == 2) {
    if (rob) hipLaunchKernelGGL(m2n_t_kernel<N2>, grid, dim3(N2::NT), 0, s, a);
    else hipLaunchKernelGGL(m2n_kernel<N2>, grid, dim3(N2::NT), 0, s, a);
  } else {
    if (rob) hipLaunchKernelGGL(m2n_t_kernel<N0>, grid, dim3(N0::NT), 0, s, a);
    else hipLaunchKernelGGL(m2n_kernel<N0>, grid, dim3(N0::NT), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_mfma2n_batched(int precision, int variant, const MfmaLaunch* descs,
                                 const int4* items, int n_items, int grid, hipStream_t s,
                                 bool robust) {
  if (n_items <= 0) return hipSuccess;
  if (precision == EM_BF16_SPLIT) {
    if (variant == 1) {
      if (robust) hipLaunchKernelGGL((m2n_batched<NB1, true>), dim3(grid), dim3(NB1::NT), 0, s, descs, items, n_items);
      else hipLaunchKernelGGL((m2n_batched<NB1, false>), dim3(grid), dim3(NB1::NT), 0, s, descs, items, n_items);
    } else {
      if (robust) hipLaunchKernelGGL((m2n_batched<NB0, true>), dim3(grid), dim3(NB0::NT), 0, s, descs, items, n_items);
      else hipLaunchKernelGGL((m2n_batched<NB0, false>), dim3(grid), dim3(NB0::NT), 0, s, descs, items, n_items);
    }
    return hipGetLastError();
  }
  if (precision != EM_FP16_SPLIT) return hipErrorInvalidValue;
  if (variant == 1) {
    if (robust) hipLaunchKernelGGL((m2n_batched<N1, true>), dim3(grid), dim3(N1::NT), 0, s, descs, items, n_items);
    else hipLaunchKernelGGL((m2n_batched<N1, false>), dim3(grid), dim3(N1::NT), 0, s, descs, items, n_items);
  } else if (variant == 2) {
    if (robust) hipLaunchKernelGGL((m2n_batched<N2, true>), dim3(grid), dim3(N2::NT), 0, s, descs, items, n_items);
    else hipLaunchKernelGGL((m2n_batched<N2, false>), dim3(grid), dim3(N2::NT), 0, s, descs, items, n_items);
  } else {
    if (robust) hipLaunchKernelGGL((m2n_batched<N0, true>), dim3(grid), dim3(N0::NT), 0, s, descs, items, n_items);
    else hipLaunchKernelGGL((m2n_batched<N0, false>), dim3(grid), dim3(N0::NT), 0, s, descs, items, n_items);
  }
  return hipGetLastError();
}

}  // namespace em
