// em_mfma2.hip -- matrix-core (MFMA) forms of the two convolutions of one EM
// iteration with super-resolution factor 2 (arXiv:2302.05804, Sec. 2,
// Eq. (3) and Eq. (2)).
//
// With k = h * 1_{2x2} (the (K+1) x (K+1) kernel of the 2x2 box sum of
// h * x read at stride 2; K = 43, K+1 = 44, c+1 = 22):
//   forward  m[I][J] = sum_{a,b} g[a][b] x[2I - 21 + a][2J - 21 + b],  g = k flipped,
//   adjoint  s[k][l] = sum_{I,J} r[I][J] k[2I + 22 - k][2J + 22 - l].
//
// Forward: output blocks of 16 x 16 frame pixels.  For each kernel row a the
// sum over b is a product with a stride-2 banded Toeplitz matrix,
//   O += X_a(16 x 96) . U_a(96 x 16),  X_a[i][p] = x[2(I0+i) - 21 + a][2 J0 - 21 + p],
//   U_a[p][j] = g[a][p - 2j]  (0 <= p - 2j < 44),
// three v_mfma_f32_16x16x32_bf16 k-chunks per row (44 of 96 p-values of a
// column are non-zero).  Rows a = r + 32 m share A fragments across block rows.
//
// Adjoint: output rows are split by parity q (k = 2i + q).  For each parity the
// sum is a 22-tap correlation on the frame grid,
//   s[2i+q][l] = sum_{alpha,J} k[2 alpha + q][2J + 22 - l] r[i + alpha + q - 11][J],
// and for 16 consecutive latent columns the column sum is one Toeplitz product
// within a single 32-wide k-chunk: U[p][j] = k[2 alpha + q][2p - j].  A fragment
// of r rows (sigma + i) serves parity 0 with alpha = sigma - 16 beta and parity 1
// with alpha - 1, so one LDS read feeds both output parities.
//
// Precision encodings and data movement as for sr = 1 (em_mfma.hip): operand
// encodings of em_mfma_common.h, FP32 accumulation; input tile in LDS, one
// plane per image part; Toeplitz fragments pre-built per frame in MFMA lane
// order, followed by the frames' scale exponents for scaled encodings.
#include "em_device.h"
#include "em_internal.h"
#include "em_mfma_common.h"

#include <type_traits>

namespace em {

constexpr int M2_KC = 44;        // box-extended kernel size for K = 43
constexpr int M2_FROWS = 64;     // forward table rows (44 used, 2 classes of 32)
constexpr int M2_FCH = 3;        // forward k-chunks per kernel row
constexpr int M2_AROWS = 32;     // adjoint table rows per parity (22 used)
constexpr int M2_FTILE = 64;     // forward: 64 x 64 frame pixels per workgroup (two image planes)
// the one-plane binary16 form takes 128 x 64 frame pixels: 2 x 2 blocks per wave
// halve the Toeplitz fragments read from LDS per product
constexpr int M2_FTILE_H16 = 128;
template <int PREC>
constexpr int m2f_tile_h() { return PREC == EM_FP16_SPLIT ? M2_FTILE_H16 : M2_FTILE; }
constexpr int M2_ATILE = 128;    // adjoint: 128 x 128 latent pixels per workgroup
// the one-plane binary16 form: 128 x 256 latent pixels, so that 8 waves own 2 x 4
// (or 4 x 2, 1 x 8) blocks and a class's Toeplitz fragments feed more products
constexpr int M2_ATILE_W16 = 256;
template <int PREC>
constexpr int m2a_tile_w() { return PREC == EM_FP16_SPLIT ? M2_ATILE_W16 : M2_ATILE; }
// bytes of one frame's fragment tables (16-byte fragments, 64 lanes)
constexpr size_t M2_FWD_FRAME_BYTES = (size_t)M2_FROWS * M2_FCH * 2 * 64 * 16;
constexpr size_t M2_ADJ_FRAME_BYTES = (size_t)2 * M2_AROWS * 2 * 64 * 16;

// Scale exponents of the frames (scaled encodings): n ints after the fragments.
__device__ inline const int* m2_table_exponents(const MfmaLaunch& a, size_t frame_bytes) {
  return reinterpret_cast<const int*>(static_cast<const char*>(a.tab) + (size_t)a.n * frame_bytes);
}

// ---------------------------------------------------------------------------
// forward, sr = 2
// ---------------------------------------------------------------------------
// PFT = 1: each wave prefetches the next class's Toeplitz fragments into
// registers; PFT = 2: the workgroup stages them in LDS (two buffers, one
// barrier per class), as for sr = 1.
template <int PREC_, int BR_, int BC_, int WR_, int WC_, int PFT_>
struct M2F {
  using P = Prec<PREC_>;
  using frag = typename P::frag;
  static constexpr int PREC = PREC_, BR = BR_, BC = BC_, WR = WR_, WC = WC_, PFT = PFT_;
  static constexpr int NS = P::NP, NA = P::NA, NB = P::NB;
  static constexpr int NTF = 2 * M2_FCH * NB;   // Toeplitz fragments of one class
  static constexpr int NW = WR * WC, NT = 64 * NW;
  static constexpr int TH = 16 * BR * WR, TW = 16 * BC * WC;      // frame pixels
  static constexpr int ROWS = 2 * TH + M2_KC - 2;                   // latent rows staged
  static constexpr int COLS = 2 * TW + 64;                          // latent cols staged
  static constexpr int PITCH = mf_pitch(COLS, 2);   // fragment rows are 2 apart
  // FP16 split: the lo part of the PSF on the 22 rows a = 11..32 of the 44-row
  // box-extended kernel only (the core; the hi part alone elsewhere)
  static constexpr bool BAND = PREC_ == EM_FP16_SPLIT;
};

// kernel rows of the 44 x 44 box-extended kernel that take the PSF's lo part
// in the FP16 split form
__host__ __device__ constexpr bool m2_lo_row(int a) { return a >= 11 && a <= 32; }

template <class C>
__device__ inline void m2f_load_T(typename C::frag (&T)[2][M2_FCH][C::NB],
                                  const typename C::frag* __restrict__ tab_t, int r) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int h = 0; h < M2_FCH; ++h)
#pragma unroll
      for (int s = 0; s < C::NB; ++s)
        T[m][h][s] = tab_t[(((r + 32 * m) * M2_FCH + h) * 2 + s) * 64 + lane];
}

// one tap class a = r + 32 m (m < NM); member m takes the PSF's lo part when
// bit m of LOM is set
template <class C, int NM, int LOM = 3>
__device__ inline void m2f_class(int r, const unsigned short (*sh)[C::ROWS * C::PITCH],
                                 const typename C::frag (&T)[2][M2_FCH][C::NB], int row_base,
                                 int col_base, f32x4 (&acc)[C::BR][C::BC]) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  constexpr int NRHO = C::BR + NM - 1;
  constexpr int NK = C::BC + M2_FCH - 1;
#pragma unroll
  for (int rho = 0; rho < NRHO; ++rho) {
    const int lrow = row_base + r + 32 * rho + 2 * i;
    typename C::frag A[NK][C::NA];
#pragma unroll
    for (int kap = 0; kap < NK; ++kap) {
      const int o = lrow * C::PITCH + col_base + 32 * kap + 8 * g;
#pragma unroll
      for (int p = 0; p < C::NA; ++p)
        A[kap][p] = *reinterpret_cast<const typename C::frag*>(&sh[p][o]);
    }
#pragma unroll
    for (int s = 0; s < C::NS; ++s)
#pragma unroll
      for (int kap = 0; kap < NK; ++kap)
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          const int beta = rho - m;
          if (beta < 0 || beta >= C::BR) continue;
          if (C::P::pb(s) == 1 && !((LOM >> m) & 1)) continue;   // no lo term on this row
#pragma unroll
          for (int h = 0; h < M2_FCH; ++h) {
            const int gam = kap - h;
            if (gam < 0 || gam >= C::BC) continue;
            acc[beta][gam] =
                C::P::mma(A[kap][C::P::pa(s)], T[m][h][C::P::pb(s)], acc[beta][gam]);
          }
        }
  }
}

// LDS buffers of the Toeplitz fragments (PFT = 2) and what the bodies allocate.
template <class C>
using M2TBuf = typename C::frag[2][C::NTF][64];
template <class C>
using M2TBufDecl = std::conditional_t<C::PFT == 2, M2TBuf<C>, int[4]>;

// Forward class r: buffer fragment f = (m, h, s) is table fragment
// ((r + 32 m) FCH + h) 2 + s.
template <class C>
__device__ inline void m2f_issue_T(const typename C::frag* __restrict__ tab_t, int r, void* dst) {
  stage_frags<C::NTF, C::NW>(
      tab_t,
      [r](int f) {
        const int s = f % C::NB, h = (f / C::NB) % M2_FCH, m = f / (C::NB * M2_FCH);
        return ((r + 32 * m) * M2_FCH + h) * 2 + s;
      },
      dst);
}

// All 32 forward classes of one frame with LDS-staged fragments (on entry class
// 0 is in buffer step & 1); the last class starts the copy of the next frame's
// class 0 when tab_next is given.
template <class C>
__device__ inline void m2f_frame_lds(const unsigned short (*sh)[C::ROWS * C::PITCH],
                                     const typename C::frag* __restrict__ tab_t,
                                     const typename C::frag* __restrict__ tab_next,
                                     M2TBuf<C>& tl, int& step, int row_base, int col_base,
                                     f32x4 (&acc)[C::BR][C::BC]) {
  const int lane = threadIdx.x & 63;
#pragma unroll 1
  for (int r = 0; r < 32; ++r) {
    const int cur = step & 1;
    if (r + 1 < 32) m2f_issue_T<C>(tab_t, r + 1, (void*)&tl[cur ^ 1][0][0]);
    else if (tab_next != nullptr) m2f_issue_T<C>(tab_next, 0, (void*)&tl[cur ^ 1][0][0]);
    // the Toeplitz fragments of the class's members (2 for r < 12, else 1)
    typename C::frag Tc[2][M2_FCH][C::NB];
    auto read_T = [&](int nm) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < M2_FCH; ++h)
#pragma unroll
          for (int q = 0; q < C::NB; ++q)
            if (m < nm) Tc[m][h][q] = tl[cur][(m * M2_FCH + h) * C::NB + q][lane];
    };
    if constexpr (C::BAND) {
      // rows r and r + 32 against the lo band 11..32: r = 0 -> (no, yes);
      // 1..10 -> (no, no); 11 -> (yes, no); 12..31 -> (yes)
      static_assert(!m2_lo_row(0) && m2_lo_row(32) && !m2_lo_row(10) && !m2_lo_row(42) &&
                        m2_lo_row(11) && !m2_lo_row(43) && m2_lo_row(12) && m2_lo_row(31),
                    "class segments follow the lo band");
      if (r == 0) {
        read_T(2);
        m2f_class<C, 2, 2>(r, sh, Tc, row_base, col_base, acc);
      } else if (r < 11) {
        read_T(2);
        m2f_class<C, 2, 0>(r, sh, Tc, row_base, col_base, acc);
      } else if (r == 11) {
        read_T(2);
        m2f_class<C, 2, 1>(r, sh, Tc, row_base, col_base, acc);
      } else {
        read_T(1);
        m2f_class<C, 1, 1>(r, sh, Tc, row_base, col_base, acc);
      }
    } else if (r < M2_KC - 32) {
      read_T(2);
      m2f_class<C, 2>(r, sh, Tc, row_base, col_base, acc);
    } else {
      read_T(1);
      m2f_class<C, 1>(r, sh, Tc, row_base, col_base, acc);
    }
    frags_landed();
    ++step;
  }
}

template <class C, bool ROB = false>
__device__ inline void m2f_body(const MfmaLaunch& a, const int tile, const int group) {
  __shared__ __align__(16) unsigned short sh[C::NA][C::ROWS * C::PITCH];
  __shared__ double red[C::NW];
  __shared__ float redf[C::NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w / C::WC, wc = w % C::WC;
  const int tiles_x = (a.W + C::TW - 1) / C::TW;      // a.H, a.W: frame grid
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int I0 = ty * C::TH, J0 = tx * C::TW;
  const int Hl = 2 * a.H, Wl = 2 * a.W;
  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const typename C::frag* tab = reinterpret_cast<const typename C::frag*>(a.tab);
  constexpr int64_t TSTRIDE = (int64_t)M2_FROWS * M2_FCH * 2 * 64;   // fragments per frame
  __shared__ __align__(16) M2TBufDecl<C> tl;
  int step = 0;
  if constexpr (C::PFT == 2) m2f_issue_T<C>(tab + t0 * TSTRIDE, 0, (void*)&tl[0][0][0]);
  const int sx = stage_tile<C::PREC, C::ROWS, C::COLS, C::PITCH, C::NT>(
      a.in, Hl, Wl, 2 * I0 - 21, 2 * J0 - 21, sh, redf);
  if constexpr (C::PFT == 2) frags_landed();
  else __syncthreads();
  const int row_base = wr * 32 * C::BR;    // latent rows of this wave's block row 0
  const int col_base = wc * 32 * C::BC;    // latent cols
  const int64_t N = (int64_t)a.H * a.W;
  double llp = 0.0;
  for (int t = t0; t < t1; ++t) {
    __asm__ volatile("" ::: "memory");   // keep tile reads inside the frame loop
    f32x4 acc[C::BR][C::BC];
#pragma unroll
    for (int b = 0; b < C::BR; ++b)
#pragma unroll
      for (int q = 0; q < C::BC; ++q) acc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const typename C::frag* tab_t = tab + t * TSTRIDE;
    if constexpr (C::PFT == 2) {
      m2f_frame_lds<C>(sh, tab_t, t + 1 < t1 ? tab_t + TSTRIDE : nullptr, tl, step, row_base,
                       col_base, acc);
    } else {
      typename C::frag Tc[2][M2_FCH][C::NB], Tn[2][M2_FCH][C::NB];
      m2f_load_T<C>(Tc, tab_t, 0);
      for (int r = 0; r < 32; ++r) {
        if (r + 1 < 32) m2f_load_T<C>(Tn, tab_t, r + 1);
        if (r < M2_KC - 32) m2f_class<C, 2>(r, sh, Tc, row_base, col_base, acc);
        else m2f_class<C, 1>(r, sh, Tc, row_base, col_base, acc);
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int h = 0; h < M2_FCH; ++h)
#pragma unroll
            for (int q = 0; q < C::NB; ++q) Tc[m][h][q] = Tn[m][h][q];
      }
    }
    const int unscale =
        C::P::SCALED ? -(sx + m2_table_exponents(a, M2_FWD_FRAME_BYTES)[t]) : 0;
    const BlockPos pos{I0 + wr * 16 * C::BR, J0 + wc * 16 * C::BC, 1};
    if constexpr (ROB) {
      llp += forward_epilogue_t<C::BR, C::BC>(acc, unscale, pos, a.H, a.W, a.u + (int64_t)t * N,
                                              a.y + (int64_t)t * N, a.out + (int64_t)t * N,
                                              a.out_y + (int64_t)t * N, a.nu, a.lcst,
                                              a.part != nullptr);
    } else {
      const float* ut = a.u ? a.u + (int64_t)t * N : nullptr;
      const float* yt = (a.u && a.part) ? a.y + (int64_t)t * N : nullptr;
      float* ot = a.out ? a.out + (int64_t)t * N : nullptr;
      llp += forward_epilogue<C::BR, C::BC>(acc, unscale, pos, a.H, a.W, ut, yt, ot);
    }
  }
  if (a.part != nullptr) {
    const double s = block_sum<C::NT>(llp, red);
    if (threadIdx.x == 0) a.part[(int64_t)group * a.ntiles + tile] = s;
  }
}

// ---------------------------------------------------------------------------
// adjoint, sr = 2
// ---------------------------------------------------------------------------
template <int PREC_, int BR_, int BC_, int WR_, int WC_, int PFT_>
struct M2A {
  using P = Prec<PREC_>;
  using frag = typename P::frag;
  static constexpr int PREC = PREC_, BR = BR_, BC = BC_, WR = WR_, WC = WC_, PFT = PFT_;
  static constexpr int NS = P::NP, NA = P::NA, NB = P::NB;
  static constexpr int NTF = 2 * 2 * NB;        // Toeplitz fragments of one class
  static constexpr int NW = WR * WC, NT = 64 * NW;
  static constexpr int THL = 32 * BR * WR, TWL = 16 * BC * WC;     // latent pixels
  // frame rows staged: THL/2 + 22 are read; the margin keeps every fragment
  // address of the unrolled class loop inside the tile
  static constexpr int ROWS = THL / 2 + 32;
  static constexpr int COLS = TWL / 2 + 24;                         // frame cols staged
  static constexpr int PITCH = mf_pitch(COLS);
  static constexpr bool BAND = PREC_ == EM_FP16_SPLIT;   // as for M2F
};

// Toeplitz fragments of adjoint class r: T[q][m] for alpha = r - q + 16 m.
template <class C>
__device__ inline void m2a_load_T(typename C::frag (&T)[2][2][C::NB],
                                  const typename C::frag* __restrict__ tab_t, int r) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      int al = r - q + 16 * m;
      al = al < 0 ? M2_AROWS - 1 : al;    // (alpha = -1 is never used; row 31 is zero)
#pragma unroll
      for (int s = 0; s < C::NB; ++s)
        T[q][m][s] = tab_t[((q * M2_AROWS + al) * 2 + s) * 64 + lane];
    }
}

// One class of the adjoint: fragment rows R + 16 rho + i (R compile-time, so the
// validity of every (parity, tap) pair folds away).
template <class C, int R>
__device__ inline void m2a_class(const unsigned short (*sh)[C::ROWS * C::PITCH],
                                 const typename C::frag (&T)[2][2][C::NB], int row_base,
                                 int col_base, f32x4 (&acc)[2][C::BR][C::BC]) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  // two-plane forms with 4-wave workgroups: the wave issuing products runs at
  // raised priority (c4 BF16 split adjoint 0.79 -> 0.73 ms; the 8-wave variant
  // loses with it)
  constexpr bool PRIO = C::NA == 2 && C::NW == 4;
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
  for (int rho = 0; rho < C::BR + 1; ++rho) {
    // skip fragment rows no (parity, tap) pair of this class uses
    bool used = false;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int beta = rho - m, al = R - q + 16 * m;
        used = used || (beta >= 0 && beta < C::BR && al >= 0 && al < 22);
      }
    if (!used) continue;
    const int lrow = row_base + R + 16 * rho + i;
    typename C::frag A[C::BC][C::NA];
#pragma unroll
    for (int gam = 0; gam < C::BC; ++gam) {
      const int o = lrow * C::PITCH + col_base + 8 * gam + 8 * g;
#pragma unroll
      for (int p = 0; p < C::NA; ++p)
        A[gam][p] = *reinterpret_cast<const typename C::frag*>(&sh[p][o]);
    }
#pragma unroll
    for (int s = 0; s < C::NS; ++s)
#pragma unroll
      for (int gam = 0; gam < C::BC; ++gam)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            // alpha = R - q + 16 m serves block row beta = rho - m
            const int beta = rho - m;
            if (beta < 0 || beta >= C::BR) continue;
            const int al = R - q + 16 * m;
            if (al < 0 || al >= 22) continue;
            // kernel row 2 alpha + q: the PSF's lo part only inside the band
            if (C::BAND && C::P::pb(s) == 1 && !m2_lo_row(2 * al + q)) continue;
            acc[q][beta][gam] =
                C::P::mma(A[gam][C::P::pa(s)], T[q][m][C::P::pb(s)], acc[q][beta][gam]);
          }
  }
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
}

// Classes R .. 15 with the next class's Toeplitz fragments fetched early.
template <class C, int R>
__device__ inline void m2a_classes(const unsigned short (*sh)[C::ROWS * C::PITCH],
                                   const typename C::frag* __restrict__ tab_t,
                                   typename C::frag (&Tc)[2][2][C::NB], int row_base,
                                   int col_base, f32x4 (&acc)[2][C::BR][C::BC]) {
  if constexpr (R < 16) {
    typename C::frag Tn[2][2][C::NB];
    if constexpr (R + 1 < 16) m2a_load_T<C>(Tn, tab_t, R + 1);
    m2a_class<C, R>(sh, Tc, row_base, col_base, acc);
    if constexpr (R + 1 < 16) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int s = 0; s < C::NB; ++s) Tc[q][m][s] = Tn[q][m][s];
      m2a_classes<C, R + 1>(sh, tab_t, Tc, row_base, col_base, acc);
    }
  }
}

// Adjoint class r: buffer fragment f = (q, m, s) is table fragment
// (q AROWS + alpha) 2 + s with alpha = r - q + 16 m (alpha = -1 -> the zero row).
template <class C>
__device__ inline void m2a_issue_T(const typename C::frag* __restrict__ tab_t, int r, void* dst) {
  stage_frags<C::NTF, C::NW>(
      tab_t,
      [r](int f) {
        const int s = f % C::NB, m = (f / C::NB) % 2, q = f / (2 * C::NB);
        int al = r - q + 16 * m;
        al = al < 0 ? M2_AROWS - 1 : al;
        return (q * M2_AROWS + al) * 2 + s;
      },
      dst);
}

// Adjoint classes R .. 15 with LDS-staged fragments (class R in buffer
// step & 1 on entry).
template <class C, int R>
__device__ inline void m2a_classes_lds(const unsigned short (*sh)[C::ROWS * C::PITCH],
                                       const typename C::frag* __restrict__ tab_t,
                                       const typename C::frag* __restrict__ tab_next,
                                       M2TBuf<C>& tl, int& step, int row_base, int col_base,
                                       f32x4 (&acc)[2][C::BR][C::BC]) {
  if constexpr (R < 16) {
    const int lane = threadIdx.x & 63;
    const int cur = step & 1;
    if constexpr (R + 1 < 16) m2a_issue_T<C>(tab_t, R + 1, (void*)&tl[cur ^ 1][0][0]);
    else if (tab_next != nullptr) m2a_issue_T<C>(tab_next, 0, (void*)&tl[cur ^ 1][0][0]);
    typename C::frag Tc[2][2][C::NB];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int s = 0; s < C::NB; ++s) Tc[q][m][s] = tl[cur][(q * 2 + m) * C::NB + s][lane];
    m2a_class<C, R>(sh, Tc, row_base, col_base, acc);
    frags_landed();
    ++step;
    m2a_classes_lds<C, R + 1>(sh, tab_t, tab_next, tl, step, row_base, col_base, acc);
  }
}

template <class C>
__device__ inline void m2a_body(const MfmaLaunch& a, const int tile, const int group) {
  __shared__ __align__(16) unsigned short sh[C::NA][C::ROWS * C::PITCH];
  __shared__ double red[2 * C::NW];
  __shared__ float redf[C::NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w / C::WC, wc = w % C::WC;
  const int Hf = a.H / 2, Wf = a.W / 2;             // a.H, a.W: latent grid
  const int tiles_x = (a.W + C::TWL - 1) / C::TWL;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int K0 = ty * C::THL, L0 = tx * C::TWL;     // both even
  const int64_t Nf = (int64_t)Hf * Wf;
  const int64_t Nl = (int64_t)a.H * a.W;
  const int row_base = wr * 16 * C::BR;             // frame rows (relative to K0/2 - 11)
  const int col_base = wc * 8 * C::BC;              // frame cols (relative to L0/2 - 11)

  f32x4 acc[2][C::BR][C::BC];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int b = 0; b < C::BR; ++b)
#pragma unroll
      for (int c2 = 0; c2 < C::BC; ++c2) acc[q][b][c2] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const typename C::frag* tab = reinterpret_cast<const typename C::frag*>(a.tab);
  constexpr int64_t TSTRIDE = (int64_t)2 * M2_AROWS * 2 * 64;   // fragments per frame
  __shared__ __align__(16) M2TBufDecl<C> tl;
  int step = 0;
  if constexpr (C::PFT == 2) m2a_issue_T<C>(tab + t0 * TSTRIDE, 0, (void*)&tl[0][0][0]);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();
    // one pixel pair at a time: batched loads made two of the three BF16 split
    // variants 45% slower here
    const int sr_t = stage_tile<C::PREC, C::ROWS, C::COLS, C::PITCH, C::NT, 0>(
        a.in + (int64_t)t * Nf, Hf, Wf, K0 / 2 - 11, L0 / 2 - 11, sh, redf);
    if constexpr (C::PFT == 2) frags_landed();
    else __syncthreads();
    const typename C::frag* tab_t = tab + t * TSTRIDE;
    const typename C::frag* tab_next = t + 1 < t1 ? tab_t + TSTRIDE : nullptr;
    // classes r = 0..15 (fragment rows r + 16 rho) cover every (parity, tap) once
    typename C::frag Tc[2][2][C::NB];
    if constexpr (C::PFT != 2) m2a_load_T<C>(Tc, tab_t, 0);
    if constexpr (C::P::SCALED) {
      // per-frame accumulators, added to the total with both scales removed
      f32x4 accf[2][C::BR][C::BC];
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int b = 0; b < C::BR; ++b)
#pragma unroll
          for (int c2 = 0; c2 < C::BC; ++c2) accf[q][b][c2] = f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (C::PFT == 2)
        m2a_classes_lds<C, 0>(sh, tab_t, tab_next, tl, step, row_base, col_base, accf);
      else
        m2a_classes<C, 0>(sh, tab_t, Tc, row_base, col_base, accf);
      const int unscale = -(sr_t + m2_table_exponents(a, M2_ADJ_FRAME_BYTES)[t]);
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int b = 0; b < C::BR; ++b)
#pragma unroll
          for (int c2 = 0; c2 < C::BC; ++c2)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[q][b][c2][v] += ldexpf(accf[q][b][c2][v], unscale);
    } else {
      (void)sr_t;
      if constexpr (C::PFT == 2)
        m2a_classes_lds<C, 0>(sh, tab_t, tab_next, tl, step, row_base, col_base, acc);
      else
        m2a_classes<C, 0>(sh, tab_t, Tc, row_base, col_base, acc);
    }
  }

  double dsq = 0.0, xsq = 0.0;
  float* pl = a.fused ? nullptr : a.plane + (int64_t)group * Nl;
  // output rows of parity q: K0 + 2 (16 b + 4 (lane / 16) + v) + q
#pragma unroll
  for (int q = 0; q < 2; ++q)
    adjoint_epilogue<C::BR, C::BC>(acc[q],
                                   BlockPos{K0 + 2 * wr * 16 * C::BR + q, L0 + wc * 16 * C::BC, 2},
                                   a.H, a.W, a.fused, a.x, a.B, pl, dsq, xsq);
  if (a.fused && a.part != nullptr) {
    const double s1 = block_sum<C::NT>(dsq, red);
    __syncthreads();
    const double s2 = block_sum<C::NT>(xsq, red + C::NW);
    if (threadIdx.x == 0) {
      a.part[2 * tile] = s1;
      a.part[2 * tile + 1] = s2;
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint, sr = 2, FP16 split, on binary16 r planes
// ---------------------------------------------------------------------------
// The forward with the frames in N writes 2^e16[t] r_t as binary16 into frame
// t's plane at plane pixel (I + 11, J + 11), zero elsewhere, so the window of a
// latent tile (ROWS frame rows of PITCH halves from frame (K0/2 - 11, L0/2 - 11),
// the layout the staged tile has in LDS) is ROWS runs of 2 PITCH bytes starting
// at plane (K0/2, L0/2) on 16-byte boundaries.  As in the sr = 1 adjoint, the
// window is copied straight into LDS, the next frame's into the second buffer
// during the first classes of the current frame, one copy per wave and class;
// a copy may stay in flight for one more class, since a wave's loads complete in
// issue order and each class waits only until its newest copy is the one left.
template <class C>
struct M2Win {
  static constexpr int HALVES = C::ROWS * C::PITCH;
  static constexpr int BYTES = 2 * HALVES;
  static constexpr int ROW_BYTES = 2 * C::PITCH;
  static constexpr int NCH = (BYTES + 1023) / 1024;       // 1 KB copies per window
  static constexpr int CCL = (NCH + C::NW - 1) / C::NW;   // classes that carry copies
  static_assert(ROW_BYTES % 16 == 0, "16-byte pieces never straddle window rows");
  static_assert(CCL < 16, "the last class of a frame carries no copy, so its wait completes the window");
};

template <class C>
__device__ inline void m2_copy_window_chunk(const unsigned short* __restrict__ plane, int p16,
                                            int k0, int l0, int ch, unsigned short* dst) {
  using Wn = M2Win<C>;
  const int o = ch * 1024 + 16 * (threadIdx.x & 63);
  if (o < Wn::BYTES) {
    const int row = o / Wn::ROW_BYTES, cb = o - row * Wn::ROW_BYTES;
    const char* src =
        reinterpret_cast<const char*>(plane + (int64_t)(k0 + row) * p16 + l0) + cb;
    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src),
                                     (__attribute__((address_space(3))) void*)(
                                         reinterpret_cast<char*>(dst) + ch * 1024),
                                     16, 0, 0);
  }
}

// Classes R .. 15 of one frame: this class's fragments are read from LDS before
// the next class's fragment copy and the window copy are issued (so no wait for
// those copies lands before the products).
template <class C, int R>
__device__ inline void m2a16_classes(const unsigned short (*sh)[C::ROWS * C::PITCH],
                                     const typename C::frag* __restrict__ tab_t,
                                     const typename C::frag* __restrict__ tab_next,
                                     M2TBuf<C>& tl, int& step, int row_base, int col_base,
                                     f32x4 (&acc)[2][C::BR][C::BC],
                                     const unsigned short* __restrict__ next_plane, int p16,
                                     int k0, int l0, unsigned short* next_buf) {
  if constexpr (R < 16) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int cur = step & 1;
    typename C::frag Tc[2][2][C::NB];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int s = 0; s < C::NB; ++s) Tc[q][m][s] = tl[cur][(q * 2 + m) * C::NB + s][lane];
    if constexpr (R + 1 < 16) m2a_issue_T<C>(tab_t, R + 1, (void*)&tl[cur ^ 1][0][0]);
    else if (tab_next != nullptr) m2a_issue_T<C>(tab_next, 0, (void*)&tl[cur ^ 1][0][0]);
    const int ch = R * C::NW + w;
    const bool copied = next_plane != nullptr && R < M2Win<C>::CCL && ch < M2Win<C>::NCH;
    if (copied) m2_copy_window_chunk<C>(next_plane, p16, k0, l0, ch, next_buf);
    m2a_class<C, R>(sh, Tc, row_base, col_base, acc);
    // s_waitcnt vmcnt(1 or 0) lgkmcnt(0): this class's fragment copies have landed
    if (copied) __builtin_amdgcn_s_waitcnt(0x0071);
    else __builtin_amdgcn_s_waitcnt(0x0070);
    __builtin_amdgcn_s_barrier();
    ++step;
    m2a16_classes<C, R + 1>(sh, tab_t, tab_next, tl, step, row_base, col_base, acc, next_plane,
                            p16, k0, l0, next_buf);
  }
}

template <class C>
__device__ inline void m2a16_body(const MfmaLaunch& a, const int tile, const int group) {
  static_assert(C::PREC == EM_FP16_SPLIT && C::PFT == 2, "r16 planes feed the FP16 split form");
  static_assert(C::ROWS == C::THL / 2 + 32 && C::PITCH == C::TWL / 2 + 48,
                "the window geometry the planes are laid out for (r16_rows, r16_pitch)");
  using Wn = M2Win<C>;
  __shared__ __align__(16) unsigned short rb[2][Wn::HALVES];
  __shared__ double red[2 * C::NW];
  __shared__ __align__(16) M2TBufDecl<C> tl;
  const int w = threadIdx.x >> 6;
  const int wr = w / C::WC, wc = w % C::WC;
  const int tiles_x = (a.W + C::TWL - 1) / C::TWL;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int K0 = ty * C::THL, L0 = tx * C::TWL;     // both even
  const int64_t Nl = (int64_t)a.H * a.W;
  const int row_base = wr * 16 * C::BR;             // frame rows (relative to K0/2 - 11)
  const int col_base = wc * 8 * C::BC;              // frame cols (relative to L0/2 - 11)

  f32x4 acc[2][C::BR][C::BC];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int b = 0; b < C::BR; ++b)
#pragma unroll
      for (int c2 = 0; c2 < C::BC; ++c2) acc[q][b][c2] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const typename C::frag* tab = reinterpret_cast<const typename C::frag*>(a.tab);
  constexpr int64_t TSTRIDE = (int64_t)2 * M2_AROWS * 2 * 64;   // fragments per frame
  const int* e_tab = m2_table_exponents(a, M2_ADJ_FRAME_BYTES);
  int step = 0;
  // first frame: its window and its first class's fragments, all waves
  m2a_issue_T<C>(tab + t0 * TSTRIDE, 0, (void*)&tl[0][0][0]);
  for (int ch = w; ch < Wn::NCH; ch += C::NW)
    m2_copy_window_chunk<C>(a.r16 + (int64_t)t0 * a.s16, a.p16, K0 / 2, L0 / 2, ch, &rb[0][0]);
  __builtin_amdgcn_s_waitcnt(0x0070);
  __builtin_amdgcn_s_barrier();
  for (int t = t0; t < t1; ++t) {
    const int buf = (t - t0) & 1;
    const unsigned short(*sh)[C::ROWS * C::PITCH] =
        reinterpret_cast<const unsigned short(*)[C::ROWS * C::PITCH]>(&rb[buf][0]);
    const bool more = t + 1 < t1;
    const unsigned short* next_plane = more ? a.r16 + (int64_t)(t + 1) * a.s16 : nullptr;
    const typename C::frag* tab_t = tab + t * TSTRIDE;
    const typename C::frag* tab_next = more ? tab_t + TSTRIDE : nullptr;
    f32x4 accf[2][C::BR][C::BC];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int b = 0; b < C::BR; ++b)
#pragma unroll
        for (int c2 = 0; c2 < C::BC; ++c2) accf[q][b][c2] = f32x4{0.f, 0.f, 0.f, 0.f};
    m2a16_classes<C, 0>(sh, tab_t, tab_next, tl, step, row_base, col_base, accf, next_plane,
                        a.p16, K0 / 2, L0 / 2, &rb[buf ^ 1][0]);
    // each frame has its own scales: add it to the total unscaled (exact)
    const int unscale = -(a.e16[t] + e_tab[t]);
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int b = 0; b < C::BR; ++b)
#pragma unroll
        for (int c2 = 0; c2 < C::BC; ++c2)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[q][b][c2][v] += ldexpf(accf[q][b][c2][v], unscale);
  }

  double dsq = 0.0, xsq = 0.0;
  float* pl = a.fused ? nullptr : a.plane + (int64_t)group * Nl;
#pragma unroll
  for (int q = 0; q < 2; ++q)
    adjoint_epilogue<C::BR, C::BC>(acc[q],
                                   BlockPos{K0 + 2 * wr * 16 * C::BR + q, L0 + wc * 16 * C::BC, 2},
                                   a.H, a.W, a.fused, a.x, a.B, pl, dsq, xsq);
  if (a.fused && a.part != nullptr) {
    const double s1 = block_sum<C::NT>(dsq, red);
    __syncthreads();
    const double s2 = block_sum<C::NT>(xsq, red + C::NW);
    if (threadIdx.x == 0) {
      a.part[2 * tile] = s1;
      a.part[2 * tile + 1] = s2;
    }
  }
}

// ---------------------------------------------------------------------------
// entry points
// ---------------------------------------------------------------------------
template <class C>
__global__ __launch_bounds__(C::NT) void m2f_kernel(MfmaLaunch a) {
  m2f_body<C>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2f_t_kernel(MfmaLaunch a) {
  m2f_body<C, true>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2a_kernel(MfmaLaunch a) {
  m2a_body<C>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2f_batched(const MfmaLaunch* __restrict__ descs,
                                                     const int4* __restrict__ items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    const MfmaLaunch d = descs[w.x];
    m2f_body<C>(d, w.y, w.z);
    __syncthreads();
  }
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2f_t_batched(const MfmaLaunch* __restrict__ descs,
                                                       const int4* __restrict__ items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    const MfmaLaunch d = descs[w.x];
    m2f_body<C, true>(d, w.y, w.z);
    __syncthreads();
  }
}
// One work item of the batched adjoint, out of line: inlined into the item loop,
// the body's accumulators and the loop state together exceed the register file.
template <class C>
__device__ __attribute__((noinline)) void m2a_item(const MfmaLaunch d, int tile, int group) {
  m2a_body<C>(d, tile, group);
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2a_batched(const MfmaLaunch* __restrict__ descs,
                                                     const int4* __restrict__ items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    m2a_item<C>(descs[w.x], w.y, w.z);
    __syncthreads();
  }
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2a16_kernel(MfmaLaunch a) {
  m2a16_body<C>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__device__ __attribute__((noinline)) void m2a16_item(const MfmaLaunch d, int tile, int group) {
  m2a16_body<C>(d, tile, group);
}
template <class C>
__global__ __launch_bounds__(C::NT) void m2a16_batched(const MfmaLaunch* __restrict__ descs,
                                                       const int4* __restrict__ items, int n) {
  for (int it = blockIdx.x; it < n; it += gridDim.x) {
    const int4 w = items[it];
    m2a16_item<C>(descs[w.x], w.y, w.z);
    __syncthreads();
  }
}

// Toeplitz tables (one block per frame and table row):
//  dir 0 (forward): [t][a < 64][h < 3][s][lane] = U_a[32h + 8(lane/16) + e][lane%16],
//                   U_a[p][j] = g[a][p - 2j], g = k flipped (a >= 44: zero);
//  dir 1 (adjoint): [t][q][alpha < 32][s][lane] = k[2 alpha + q][2p - j],
//                   p = 8(lane/16) + e, j = lane%16 (alpha >= 22: zero).
// k = 2x2-box extension of f zero-padded from K to 43.  Scaled encodings
// multiply k by 2^e_t (e_t = f16_scale_exp of max |k_t|) and store e_t as the
// t-th of n ints after the fragments of all n frames.
template <int PREC>
__global__ __launch_bounds__(384) void m2_table_kernel(const float* psf, int n, int K, int dir,
                                                       unsigned short* tab) {
  __shared__ float redf[6];
  const int t = blockIdx.x, row = blockIdx.y;
  const int off = (43 - K) / 2;
  const float* f = psf + (int64_t)t * K * K;
  auto fp = [&](int a, int b) -> float {
    const int ia = a - off, ib = b - off;
    if (ia < 0 || ia >= K || ib < 0 || ib >= K) return 0.f;
    return f[ia * K + ib];
  };
  auto kk = [&](int a, int b) -> float {   // 44 x 44 box-extended kernel
    if (a < 0 || a >= M2_KC || b < 0 || b >= M2_KC) return 0.f;
    return (fp(a - 1, b - 1) + fp(a - 1, b)) + (fp(a, b - 1) + fp(a, b));
  };
  int ex = 0;
  if constexpr (Prec<PREC>::SCALED) {
    float mx = 0.f;
    for (int i = threadIdx.x; i < M2_KC * M2_KC; i += 384)
      mx = fmaxf(mx, fabsf(kk(i / M2_KC, i % M2_KC)));
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = redf[0];
    for (int i = 1; i < 6; ++i) mx = fmaxf(mx, redf[i]);
    ex = f16_scale_exp(mx);
    if (row == 0 && threadIdx.x == 0) {
      const size_t fb = dir == 0 ? M2_FWD_FRAME_BYTES : M2_ADJ_FRAME_BYTES;
      reinterpret_cast<int*>(reinterpret_cast<char*>(tab) + (size_t)n * fb)[t] = ex;
    }
  }
  const int idx = threadIdx.x;
  if (dir == 0) {
    // row = a in [0, 64); idx = (h, s, lane) = 3 x 2 x 64
    if (idx >= M2_FCH * 2 * 64) return;
    const int lane = idx & 63, s = (idx >> 6) & 1, h = idx >> 7;
    const int j = lane & 15, gq = lane >> 4;
    unsigned short* dst =
        tab + ((((int64_t)t * M2_FROWS + row) * M2_FCH + h) * 2 + s) * 64 * 8 + lane * 8;
    for (int e = 0; e < 8; ++e) {
      const int p = 32 * h + 8 * gq + e;
      const int b = p - 2 * j;
      float gv = 0.f;
      if (row < M2_KC && b >= 0 && b < M2_KC) gv = kk(M2_KC - 1 - row, M2_KC - 1 - b);
      dst[e] = table_part<PREC>(Prec<PREC>::SCALED ? ldexpf(gv, ex) : gv, s);
    }
  } else {
    // row = q * 32 + alpha; idx = (s, lane) = 2 x 64
    if (idx >= 2 * 64) return;
    const int q = row / M2_AROWS, al = row % M2_AROWS;
    const int lane = idx & 63, s = idx >> 6;
    const int j = lane & 15, gq = lane >> 4;
    unsigned short* dst = tab + ((((int64_t)t * 2 + q) * M2_AROWS + al) * 2 + s) * 64 * 8 + lane * 8;
    for (int e = 0; e < 8; ++e) {
      const int p = 8 * gq + e;
      const int b = 2 * p - j;
      float gv = 0.f;
      if (al < 22 && b >= 0 && b < M2_KC) gv = kk(2 * al + q, b);
      dst[e] = table_part<PREC>(Prec<PREC>::SCALED ? ldexpf(gv, ex) : gv, s);
    }
  }
}

size_t mfma2_table_bytes(int n, int dir) {
  // fragments, then one scale exponent per frame
  return (size_t)n * (dir == 0 ? M2_FWD_FRAME_BYTES : M2_ADJ_FRAME_BYTES) + (size_t)n * sizeof(int);
}

hipError_t launch_mfma2_tables(const Geometry& g, const float* psf, void* tab_fwd, void* tab_adj,
                               hipStream_t s) {
  auto ker = g.precision == EM_FP16_SPLIT ? m2_table_kernel<EM_FP16_SPLIT>
                                          : m2_table_kernel<EM_BF16_SPLIT>;
  if (uses_m2n(g)) {
    const hipError_t e = launch_mfma2n_table(g, psf, tab_fwd, s);
    if (e != hipSuccess) return e;
  } else {
    hipLaunchKernelGGL(ker, dim3(g.n, M2_FROWS), dim3(384), 0, s, psf, g.n, g.K, 0,
                       static_cast<unsigned short*>(tab_fwd));
  }
  hipLaunchKernelGGL(ker, dim3(g.n, 2 * M2_AROWS), dim3(384), 0, s, psf, g.n, g.K, 1,
                     static_cast<unsigned short*>(tab_adj));
  return hipGetLastError();
}

int mfma2_fwd_tile_h(int precision) {
  return precision == EM_FP16_SPLIT ? M2_FTILE_H16 : M2_FTILE;
}
int mfma2_fwd_tile_w(int) { return M2_FTILE; }
int mfma2_adj_tile_h(int) { return M2_ATILE; }
int mfma2_adj_tile_w(int precision) {
  return precision == EM_FP16_SPLIT ? M2_ATILE_W16 : M2_ATILE;
}

namespace {
// forward variants, FP16 split (128 x 64 frame pixels): 0: 8 waves of 2x2 blocks;
// 1: 8 waves of 4x1; 2: 8 waves of 1x4.  Two-plane encodings (64 x 64): 0: 4 waves
// of 2x2 blocks; 1: 8 waves of 2x1; 2: 8 waves of 1x2.  Adjoint variants, FP16 split
// (128 x 256 latent): 0: 8 waves of 2x4 blocks (per parity); 1: 8 waves of 4x2;
// 2: 8 waves of 1x8.  Two-plane encodings (128 x 128): 0: 8 waves of 2x2; 1: 4 waves
// of 4x2; 2: 4 waves of 2x4.
template <int PREC>
hipError_t launch2(int dir, int variant, dim3 grid, bool batched, const MfmaLaunch& a,
                   const MfmaLaunch* d, const int4* it, int n, hipStream_t s, bool robust = false,
                   bool r16 = false) {
  // Toeplitz fragments staged in LDS for the one-plane binary16 image
  constexpr int PFT = PREC == EM_FP16_SPLIT ? 2 : 1;
  constexpr bool H16 = PREC == EM_FP16_SPLIT;
  using F0 = std::conditional_t<H16, M2F<PREC, 2, 2, 4, 2, PFT>, M2F<PREC, 2, 2, 2, 2, PFT>>;
  using F1 = std::conditional_t<H16, M2F<PREC, 4, 1, 2, 4, PFT>, M2F<PREC, 2, 1, 2, 4, PFT>>;
  using F2 = std::conditional_t<H16, M2F<PREC, 1, 4, 8, 1, PFT>, M2F<PREC, 1, 2, 4, 2, PFT>>;
  using A0 = std::conditional_t<H16, M2A<PREC, 2, 4, 2, 4, PFT>, M2A<PREC, 2, 2, 2, 4, PFT>>;
  using A1 = std::conditional_t<H16, M2A<PREC, 4, 2, 1, 8, PFT>, M2A<PREC, 4, 2, 1, 4, PFT>>;
  using A2 = std::conditional_t<H16, M2A<PREC, 1, 8, 4, 2, PFT>, M2A<PREC, 2, 4, 2, 2, PFT>>;
  constexpr int FTH = m2f_tile_h<PREC>();
  static_assert(F0::TH == FTH && F0::TW == M2_FTILE && F1::TH == FTH && F1::TW == M2_FTILE &&
                F2::TH == FTH && F2::TW == M2_FTILE, "fwd tile");
  constexpr int ATW = m2a_tile_w<PREC>();
  static_assert(A0::THL == M2_ATILE && A0::TWL == ATW && A1::THL == M2_ATILE && A1::TWL == ATW &&
                A2::THL == M2_ATILE && A2::TWL == ATW, "adj tile");
#define EM_M2_LAUNCH(KER, CFG)                                                          \
  do {                                                                                  \
    if (batched)                                                                        \
      hipLaunchKernelGGL(KER##_batched<CFG>, grid, dim3(CFG::NT), 0, s, d, it, n);      \
    else                                                                                \
      hipLaunchKernelGGL(KER##_kernel<CFG>, grid, dim3(CFG::NT), 0, s, a);              \
  } while (0)
  // the adjoint on binary16 r planes (FP16 split)
  if (dir == 1 && (batched ? r16 : a.r16 != nullptr)) {
    if constexpr (PREC == EM_FP16_SPLIT) {
      if (variant == 1) EM_M2_LAUNCH(m2a16, A1);
      else if (variant == 2) EM_M2_LAUNCH(m2a16, A2);
      else EM_M2_LAUNCH(m2a16, A0);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (dir == 0 && batched && robust) {
    if (variant == 1) hipLaunchKernelGGL(m2f_t_batched<F1>, grid, dim3(F1::NT), 0, s, d, it, n);
    else if (variant == 2) hipLaunchKernelGGL(m2f_t_batched<F2>, grid, dim3(F2::NT), 0, s, d, it, n);
    else hipLaunchKernelGGL(m2f_t_batched<F0>, grid, dim3(F0::NT), 0, s, d, it, n);
  } else if (dir == 0 && !batched && a.out_y != nullptr) {
    if (variant == 1) hipLaunchKernelGGL(m2f_t_kernel<F1>, grid, dim3(F1::NT), 0, s, a);
    else if (variant == 2) hipLaunchKernelGGL(m2f_t_kernel<F2>, grid, dim3(F2::NT), 0, s, a);
    else hipLaunchKernelGGL(m2f_t_kernel<F0>, grid, dim3(F0::NT), 0, s, a);
  } else if (dir == 0) {
    if (variant == 1) EM_M2_LAUNCH(m2f, F1);
    else if (variant == 2) EM_M2_LAUNCH(m2f, F2);
    else EM_M2_LAUNCH(m2f, F0);
  } else {
    if (variant == 1) EM_M2_LAUNCH(m2a, A1);
    else if (variant == 2) EM_M2_LAUNCH(m2a, A2);
    else EM_M2_LAUNCH(m2a, A0);
  }
#undef EM_M2_LAUNCH
  return hipGetLastError();
}
}  // namespace

// forward descriptors carry the frame grid, adjoint descriptors the latent grid
bool mfma2_desc_ok(const Geometry& g, int dir, int tiles, int groups, const MfmaLaunch& a) {
  if (dir == 0 && uses_m2n(g)) return mfma2n_desc_ok(g, tiles, groups, a);
  return dir == 0
      ? (a.H == g.Hf && a.W == g.Wf &&
         launch_grid_ok(tiles, groups, a.ntiles, a.n, a.fpg, a.H, a.W,
                        mfma2_fwd_tile_h(g.precision), mfma2_fwd_tile_w(g.precision)))
      : (a.H == g.Hl && a.W == g.Wl && a.H % 2 == 0 && a.W % 2 == 0 &&
         launch_grid_ok(tiles, groups, a.ntiles, a.n, a.fpg, a.H, a.W,
                        mfma2_adj_tile_h(g.precision), mfma2_adj_tile_w(g.precision)));
}

hipError_t launch_mfma2(const Geometry& g, int dir, int variant, int tiles, int groups,
                        const MfmaLaunch& a, hipStream_t s) {
  if (!mfma2_desc_ok(g, dir, tiles, groups, a)) return hipErrorInvalidValue;
  if (dir == 0 && uses_m2n(g)) return launch_mfma2n(g, variant, tiles, groups, a, s);
  dim3 grid(tiles, groups);
  switch (g.precision) {
    case EM_BF16_SPLIT: return launch2<EM_BF16_SPLIT>(dir, variant, grid, false, a, nullptr, nullptr, 0, s);
    case EM_FP16_SPLIT: return launch2<EM_FP16_SPLIT>(dir, variant, grid, false, a, nullptr, nullptr, 0, s);
    case EM_BF16: return launch2<EM_BF16>(dir, variant, grid, false, a, nullptr, nullptr, 0, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mfma2_batched(int precision, int dir, int variant, const MfmaLaunch* descs,
                                const int4* items, int n_items, int grid, hipStream_t s,
                                bool robust, bool m2n, bool r16) {
  if (n_items <= 0) return hipSuccess;
  if (m2n) {
    if (dir != 0) return hipErrorInvalidValue;
    return launch_mfma2n_batched(precision, variant, descs, items, n_items, grid, s, robust);
  }
  MfmaLaunch dummy{};
  switch (precision) {
    case EM_BF16_SPLIT: return launch2<EM_BF16_SPLIT>(dir, variant, dim3(grid), true, dummy, descs, items, n_items, s, robust);
    case EM_FP16_SPLIT: return launch2<EM_FP16_SPLIT>(dir, variant, dim3(grid), true, dummy, descs, items, n_items, s, robust, r16);
    case EM_BF16: return launch2<EM_BF16>(dir, variant, dim3(grid), true, dummy, descs, items, n_items, s, robust);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace em
