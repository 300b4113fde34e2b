// em_mfma.hip -- matrix-core (MFMA) forms of the two convolutions of one EM
// iteration (arXiv:2302.05804, Sec. 2, Eqs. (1)-(2)), sr = 1.
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
// Precision (template argument PREC, encodings in em_mfma_common.h): bf16 hi +
// lo split of both operands with three products (EM_BF16_SPLIT), plain bf16
// (EM_BF16), or a binary16 image operand with a per-tile power-of-two scale
// times a binary16 hi + lo PSF with a per-frame scale, two products
// (EM_FP16_SPLIT).  Accumulation is FP32 in the matrix core throughout.
//
// Data movement (per workgroup of 4 waves, 128 x 128 outputs, each wave 64 x 64
// = 4 x 4 blocks of 16 x 16):
//  * the input tile (128 + K - 1 rows, 176 columns) is stored in LDS as one
//    16-bit plane per image part (hi, lo for the bf16 split), row-major, with
//    the bank-conflict-free pitch of mf_pitch;
//  * taps are grouped in classes a = r + 16 m: the A fragment of rows
//    r + 16 rho + i then serves block rows beta = rho - m for every m of the
//    class, so one LDS read feeds up to 3 row blocks (and 2 column blocks);
//  * the Toeplitz fragments U_a (hi, lo) are pre-built per frame in the lane
//    order of the MFMA B operand and read from global memory (L2-resident);
//    scaled encodings keep the frame's scale exponents after the fragments.
#include "em_device.h"
#include "em_internal.h"
#include "em_mfma_common.h"

#include <algorithm>
#include <type_traits>

namespace em {

constexpr int MF_TILE = 128;   // every sr = 1 variant covers 128 x 128 outputs

// Tile configuration: each wave owns BR x BC blocks of 16 x 16 outputs, the
// workgroup WR x WC waves.
template <int KT_, int PREC_, int BR_, int BC_, int WR_, int WC_, int PFA_, int PFT_, int LB_ = -1>
struct MfCfg {
  using P = Prec<PREC_>;
  using frag = typename P::frag;
  static constexpr int KT = KT_, PREC = PREC_, BR = BR_, BC = BC_, WR = WR_, WC = WC_;
  static constexpr int NS = P::NP, NA = P::NA, NB = P::NB;
  // PFA: load the A fragments of the next fragment row before the products of
  // the current one.  PFT = 1: each wave fetches the next tap class's Toeplitz
  // fragments into registers early; PFT = 2: the workgroup stages them once in
  // LDS with direct global-to-LDS loads (two buffers, one barrier per class).
  static constexpr int PFA = PFA_, PFT = PFT_;
  static constexpr int NW = WR * WC, NT = 64 * NW;
  static constexpr int TH = 16 * BR * WR, TW = 16 * BC * WC;
  static constexpr int ROWS = TH + KT - 1;
  static constexpr int COLS = TW + 48;
  static constexpr int PITCH = mf_pitch(COLS);
  static constexpr int MMAX = (KT + 15) / 16;   // members of the largest tap class
  static constexpr int KTP = 16 * MMAX;         // table rows (zero beyond KT)
  static constexpr int NTF = MMAX * 2 * NB;     // Toeplitz fragments of one class
  static constexpr int RFULL = KT - 16 * (MMAX - 1);     // classes with MMAX members
  static constexpr int RLAST = (MMAX == 1) ? KT : 16;    // number of classes
  // K = 43, FP16 split (always) or BF16 split (LB_ = 1, for jobs whose PSFs keep
  // at most 1/16 of their mass outside the band): the lo parts enter only on the
  // 21 kernel rows within 10 of the centre (rows 11..31: member 1 of the
  // three-member classes r <= 10, both members of the classes r >= 11), where a
  // PSF keeps its core; elsewhere each tap is the product of the hi parts alone
  // (the PSF's relative error 2^-11 in binary16; in bf16 2^-9 for the PSF and
  // for the image operand each).  Bit m of lo_mask(NM): member m takes lo.
  static constexpr bool BAND =
      KT_ == 43 && (LB_ < 0 ? PREC_ == EM_FP16_SPLIT : (LB_ == 1 && PREC_ != EM_BF16));
  static constexpr int lo_mask(int nm) { return !BAND ? 7 : (nm == 3 ? 2 : 3); }
};

// LDS staging buffers of the Toeplitz fragments (PFT = 2): two classes, NTF
// fragments of 64 lanes each.
template <class C>
using TBuf = typename C::frag[2][C::NTF][64];
// what the kernel bodies allocate (a token when the fragments are not staged)
template <class C>
using TBufDecl = std::conditional_t<C::PFT == 2, TBuf<C>, int[4]>;

// Toeplitz fragments of tap class r (rows a = r + 16 m, m < MMAX), both k-halves,
// hi and (split) lo parts.
template <class C>
__device__ inline void load_T(typename C::frag (&T)[C::MMAX][2][C::NB],
                              const typename C::frag* __restrict__ tab_t, int r) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int m = 0; m < C::MMAX; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int s = 0; s < C::NB; ++s)
        T[m][h][s] = tab_t[(((r + 16 * m) * 2 + h) * 2 + s) * 64 + lane];
}

// A fragments (every image part) of fragment row rho for every column
// position kappa.
template <class C>
__device__ inline void load_A(typename C::frag (&A)[C::BC + 2][C::NA], const unsigned short (*sh)[C::ROWS * C::PITCH],
                              int lrow, int col_base) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int kap = 0; kap < C::BC + 2; ++kap) {
    const int o = lrow * C::PITCH + col_base + 16 * kap + 8 * g;
#pragma unroll
    for (int p = 0; p < C::NA; ++p) A[kap][p] = *reinterpret_cast<const typename C::frag*>(&sh[p][o]);
  }
}

// One tap class: NM members a = r + 16 m.  The A fragment of rows
// r + 16 rho + i serves block rows beta = rho - m; fragments of the next rho
// are loaded before the products of the current one are issued, and products
// are ordered by split term so that consecutive MFMAs write different blocks.
template <class C, int NM>
__device__ inline void mfma_class(int r, const unsigned short (*sh)[C::ROWS * C::PITCH],
                                  const typename C::frag (&T)[C::MMAX][2][C::NB], int row_base,
                                  int col_base, f32x4 (&acc)[C::BR][C::BC]) {
  const int i = threadIdx.x & 15;
  constexpr int NRHO = C::BR + NM - 1;
  constexpr int LOM = C::lo_mask(NM);
  typename C::frag A[C::PFA ? 2 : 1][C::BC + 2][C::NA];
  if (C::PFA) load_A<C>(A[0], sh, row_base + r + i, col_base);
  // two-plane forms: the wave issuing products runs at raised priority (3% off
  // the BF16 split adjoint on c3; no gain for the binary16 form)
  constexpr bool PRIO = C::NA == 2;
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
  for (int rho = 0; rho < NRHO; ++rho) {
    if (C::PFA) {
      if (rho + 1 < NRHO)
        load_A<C>(A[(rho + 1) & 1], sh, row_base + r + 16 * (rho + 1) + i, col_base);
    } else {
      load_A<C>(A[0], sh, row_base + r + 16 * rho + i, col_base);
    }
    const int cur = C::PFA ? (rho & 1) : 0;
#pragma unroll
    for (int s = 0; s < C::NS; ++s) {
#pragma unroll
      for (int kap = 0; kap < C::BC + 2; ++kap) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          const int beta = rho - m;
          if (beta < 0 || beta >= C::BR) continue;
          // outside the band: the hi x hi product alone
          if ((C::P::pa(s) == 1 || C::P::pb(s) == 1) && !((LOM >> m) & 1)) continue;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int gam = kap - 2 * h;
            if (gam < 0 || gam >= C::BC) continue;
            acc[beta][gam] = C::P::mma(A[cur][kap][C::P::pa(s)], T[m][h][C::P::pb(s)],
                                       acc[beta][gam]);
          }
        }
      }
    }
  }
  if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
}

// No prefetch of the next frame's tile (the default hook of mfma_frame).
struct NoTilePf {
  __device__ void issue() {}
};

// All kernel rows of one frame; the Toeplitz fragments of the next class are
// fetched while the current class runs.  With use_pf, pf.issue() runs after
// class 0's fragment loads and before class 1's, so class 0's products cover
// the latency of its loads.
template <class C, class PF>
__device__ __attribute__((always_inline)) inline void mfma_frame(
    const unsigned short (*sh)[C::ROWS * C::PITCH],
    const typename C::frag* __restrict__ tab_t, int row_base, int col_base,
    f32x4 (&acc)[C::BR][C::BC], PF& pf, bool use_pf) {
  // classes with MMAX members first, then MMAX-1 (KT = 43: r <= 10 -> 3, r >= 11 -> 2;
  // KT = 15: r <= 14 -> 1)
  constexpr int RFULL = C::KT - 16 * (C::MMAX - 1);
  constexpr int RLAST = (C::MMAX == 1) ? C::KT : 16;
  typename C::frag Tc[C::MMAX][2][C::NB];
  if (C::PFT) {
    typename C::frag Tn[C::MMAX][2][C::NB];
    load_T<C>(Tc, tab_t, 0);
    if (use_pf) pf.issue();
    int r = 0;
#pragma unroll 1
    for (; r < RFULL; ++r) {
      if (r + 1 < RLAST) load_T<C>(Tn, tab_t, r + 1);
      mfma_class<C, C::MMAX>(r, sh, Tc, row_base, col_base, acc);
#pragma unroll
      for (int m = 0; m < C::MMAX; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < C::NB; ++q) Tc[m][h][q] = Tn[m][h][q];
    }
    if constexpr (C::MMAX > 1) {
#pragma unroll 1
      for (; r < RLAST; ++r) {
        if (r + 1 < RLAST) load_T<C>(Tn, tab_t, r + 1);
        mfma_class<C, C::MMAX - 1>(r, sh, Tc, row_base, col_base, acc);
#pragma unroll
        for (int m = 0; m < C::MMAX; ++m)
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int q = 0; q < C::NB; ++q) Tc[m][h][q] = Tn[m][h][q];
      }
    }
  } else {
    int r = 0;
    for (; r < RFULL; ++r) {
      load_T<C>(Tc, tab_t, r);
      mfma_class<C, C::MMAX>(r, sh, Tc, row_base, col_base, acc);
    }
    if constexpr (C::MMAX > 1) {
      for (; r < RLAST; ++r) {
        load_T<C>(Tc, tab_t, r);
        mfma_class<C, C::MMAX - 1>(r, sh, Tc, row_base, col_base, acc);
      }
    }
  }
}

// PFT = 2: start copying the Toeplitz fragments of class r of one frame's
// table into an LDS buffer: buffer fragment f = (m, h, s) of the class; the
// waves of the workgroup share the fragments round robin, each lane moving its
// own 16 bytes (global_load_lds_dwordx4: destination = wave-uniform base + 16
// bytes per lane, the fragment's lane order).
template <class C>
__device__ inline void issue_T(const typename C::frag* __restrict__ tab_t, int r, void* dst_v) {
  typename C::frag* dst = static_cast<typename C::frag*>(dst_v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int f = w; f < C::NTF; f += C::NW) {
    const int s = f % C::NB, h = (f / C::NB) % 2, m = f / (2 * C::NB);
    const typename C::frag* src = tab_t + (((r + 16 * m) * 2 + h) * 2 + s) * 64 + lane;
    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)(src),
                                     (__attribute__((address_space(3))) void*)(dst + f * 64), 16,
                                     0, 0);
  }
}

template <class C>
__device__ inline int issue_u(const UPre& u, int r) {
  static_assert(C::RLAST >= 14, "the copy needs tap classes 1..13");
  return issue_u_tile<C::TH, C::TW, C::NW>(u, r);
}

// One tap class with the Toeplitz fragments staged in LDS: start the copy of
// the next class (the first class of tab_next after the last one, if any) into
// the other buffer, read this class's fragments from LDS, issue its products,
// then wait for this wave's fragment copies and meet the other waves at a
// barrier, after which the next buffer is complete and this one free.  The
// weight copies issued after the fragment copies may stay in flight into the
// next class (a wave's loads complete in issue order); the classes without a
// weight copy wait for everything, so the copies have landed by the epilogue.
template <class C, int NM>
__device__ inline void mfma_class_lds(int r, const unsigned short (*sh)[C::ROWS * C::PITCH],
                                      const typename C::frag* __restrict__ tab_t,
                                      const typename C::frag* __restrict__ tab_next,
                                      TBuf<C>& tl, int& step, int row_base, int col_base,
                                      f32x4 (&acc)[C::BR][C::BC], const UPre& up) {
  const int lane = threadIdx.x & 63;
  const int cur = step & 1;
  if (r + 1 < C::RLAST) issue_T<C>(tab_t, r + 1, (void*)&tl[cur ^ 1][0][0]);
  else if (tab_next != nullptr) issue_T<C>(tab_next, 0, (void*)&tl[cur ^ 1][0][0]);
  const int nu = __builtin_amdgcn_readfirstlane(issue_u<C>(up, r));   // wave-uniform
  typename C::frag Tc[C::MMAX][2][C::NB];
#pragma unroll
  for (int m = 0; m < C::MMAX; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < C::NB; ++q) Tc[m][h][q] = tl[cur][(m * 2 + h) * C::NB + q][lane];
  mfma_class<C, NM>(r, sh, Tc, row_base, col_base, acc);
  // s_waitcnt vmcnt(nu) lgkmcnt(0)
  if (nu == 0) __builtin_amdgcn_s_waitcnt(0x0070);
  else if (nu == 1) __builtin_amdgcn_s_waitcnt(0x0071);
  else __builtin_amdgcn_s_waitcnt(0x0072);
  // a bare barrier (a fence here would make the compiler wait for every copy),
  // and no compiler motion of memory accesses across it
  __builtin_amdgcn_s_barrier();
  __asm__ volatile("" ::: "memory");
  ++step;
}

// All classes of one frame with the Toeplitz fragments staged in LDS.  On entry
// the fragments of class 0 are in buffer step & 1 (a barrier after their copy
// has been passed).  PEEL: class 0 outside the class loop, so that waits the
// compiler places for loads still in flight from the previous frame's
// epilogue land in class 0 only, not in every class of the loop.
template <class C, bool PEEL = false>
__device__ inline void mfma_frame_lds(const unsigned short (*sh)[C::ROWS * C::PITCH],
                                      const typename C::frag* __restrict__ tab_t,
                                      const typename C::frag* __restrict__ tab_next,
                                      TBuf<C>& tl, int& step, int row_base, int col_base,
                                      f32x4 (&acc)[C::BR][C::BC],
                                      const UPre& up = UPre{nullptr, nullptr, 0, 0, 0, 0}) {
  int r = 0;
  if constexpr (PEEL) {
    mfma_class_lds<C, C::MMAX>(0, sh, tab_t, tab_next, tl, step, row_base, col_base, acc, up);
    r = 1;
  }
#pragma unroll 1
  for (; r < C::RFULL; ++r)
    mfma_class_lds<C, C::MMAX>(r, sh, tab_t, tab_next, tl, step, row_base, col_base, acc, up);
  if constexpr (C::MMAX > 1) {
#pragma unroll 1
    for (; r < C::RLAST; ++r)
      mfma_class_lds<C, C::MMAX - 1>(r, sh, tab_t, tab_next, tl, step, row_base, col_base, acc,
                                     up);
  }
}

// Scale exponents of a frame's Toeplitz table (scaled encodings): n ints after
// the fragments of all frames.
template <class C>
__device__ inline const int* table_exponents(const MfmaLaunch& a) {
  return reinterpret_cast<const int*>(static_cast<const char*>(a.tab) +
                                      (size_t)a.n * C::KTP * 4 * 64 * 16);
}

// Forward: r_t = u_t * (f_t * x) for the frames of this group, x tile staged once
// (ROB: the Student-t epilogue, which also writes u w y; R16: r written as
// binary16 into the frames' r16 planes, scaled by 2^e16[t]).
template <class C, bool ROB = false, bool R16 = false>
__device__ inline void mfma_fwd_body(const MfmaLaunch& a, const int tile, const int group) {
  static_assert(!R16 || (C::PREC == EM_FP16_SPLIT && !ROB), "r16 planes: FP16 split, Gaussian");
  constexpr int c = (C::KT - 1) / 2;
  __shared__ __align__(16) unsigned short sh[C::NA][C::ROWS * C::PITCH];
  __shared__ double red[C::NW];
  __shared__ float redf[C::NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row_base = (w / C::WC) * 16 * C::BR, col_base = (w % C::WC) * 16 * C::BC;
  const int tiles_x = (a.W + C::TW - 1) / C::TW;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int k0 = ty * C::TH, l0 = tx * C::TW;
  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const typename C::frag* tab = reinterpret_cast<const typename C::frag*>(a.tab);
  constexpr int64_t TSTRIDE = (int64_t)C::KTP * 4 * 64;   // fragments per frame
  __shared__ __align__(16) TBufDecl<C> tl;
  // u of the frame in LDS (LDS-staged fragments, plain epilogue, rows of whole 16-byte runs)
  constexpr bool UPF = C::PFT == 2 && !ROB && C::TW == 128;
  __shared__ __align__(16) std::conditional_t<UPF, float[C::TH * C::TW], float[4]> ubuf;
  const bool use_ul = UPF && a.u != nullptr && a.part == nullptr &&
                      (R16 ? a.r16 != nullptr : a.out != nullptr) && (a.W & 3) == 0 && a.W >= 4;
  int step = 0;
  if constexpr (C::PFT == 2) issue_T<C>(tab + t0 * TSTRIDE, 0, (void*)&tl[0][0][0]);
  const int sx = stage_tile<C::PREC, C::ROWS, C::COLS, C::PITCH, C::NT>(a.in, a.H, a.W, k0 - c,
                                                                        l0 - c, sh, redf);
  if constexpr (C::PFT == 2) frags_landed();
  else __syncthreads();

  const int64_t N = (int64_t)a.H * a.W;
  double llp = 0.0;
  NoTilePf no_pf;
  for (int t = t0; t < t1; ++t) {
    // The staged tile does not change between frames; this fence keeps the
    // compiler from hoisting every fragment read of the tile out of the frame
    // loop (which would need hundreds of live registers).
    __asm__ volatile("" ::: "memory");
    f32x4 acc[C::BR][C::BC];
#pragma unroll
    for (int b = 0; b < C::BR; ++b)
#pragma unroll
      for (int q = 0; q < C::BC; ++q) acc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const typename C::frag* tab_t = tab + t * TSTRIDE;
    const UPre up{use_ul ? a.u + (int64_t)t * N : nullptr, &ubuf[0], k0, l0, a.H, a.W};
    if constexpr (C::PFT == 2)
      mfma_frame_lds<C, R16>(sh, tab_t, t + 1 < t1 ? tab_t + TSTRIDE : nullptr, tl, step,
                             row_base, col_base, acc, up);
    else
      mfma_frame<C>(sh, tab_t, row_base, col_base, acc, no_pf, false);
    // exact removal of the image and PSF scales (scaled encodings)
    const int unscale = C::P::SCALED ? -(sx + table_exponents<C>(a)[t]) : 0;
    // epilogue: per-frame base pointers (wave-uniform) + 32-bit in-frame offsets
    if constexpr (R16) {
      const R16Out o{a.r16 + (int64_t)t * a.s16, a.p16, c, a.e16[t]};
      const BlockPos P{k0 + row_base, l0 + col_base, 1};
      if (UPF && use_ul)
        forward_epilogue_ul16<C::BR, C::BC, C::TW>(acc, unscale, P, a.H, a.W, k0, l0, &ubuf[0], o);
      else if (a.part != nullptr)
        llp += forward_epilogue_w16<C::BR, C::BC, true>(acc, unscale, P, a.H, a.W,
                                                        a.u + (int64_t)t * N, a.y + (int64_t)t * N, o);
      else
        (void)forward_epilogue_w16<C::BR, C::BC, false>(acc, unscale, P, a.H, a.W,
                                                        a.u + (int64_t)t * N, nullptr, o);
    } else if constexpr (ROB) {
      llp += forward_epilogue_t<C::BR, C::BC>(
          acc, unscale, BlockPos{k0 + row_base, l0 + col_base, 1}, a.H, a.W, a.u + (int64_t)t * N,
          a.y + (int64_t)t * N, a.out + (int64_t)t * N, a.out_y + (int64_t)t * N, a.nu, a.lcst,
          a.part != nullptr);
    } else if (UPF && use_ul) {
      forward_epilogue_ul<C::BR, C::BC, C::TW>(acc, unscale,
                                               BlockPos{k0 + row_base, l0 + col_base, 1}, a.H,
                                               a.W, k0, l0, &ubuf[0], a.out + (int64_t)t * N);
    } else {
      const float* ut = a.u ? a.u + (int64_t)t * N : nullptr;
      const float* yt = (a.u && a.part) ? a.y + (int64_t)t * N : nullptr;
      float* ot = a.out ? a.out + (int64_t)t * N : nullptr;
      llp += forward_epilogue<C::BR, C::BC>(acc, unscale,
                                            BlockPos{k0 + row_base, l0 + col_base, 1}, a.H, a.W,
                                            ut, yt, ot);
    }
  }
  if (a.part != nullptr) {
    const double s = block_sum<C::NT>(llp, red);
    if (threadIdx.x == 0) a.part[(int64_t)group * a.ntiles + tile] = s;
  }
}


// The next frame's r tile for the unscaled encodings (BF16 split, BF16) of the
// adjoint with register-held Toeplitz fragments: the first NPF pixel pairs per
// thread are loaded into registers during the current frame's first tap class;
// once every wave is done with the current frame, the rest are loaded in one
// batch and all are split and stored into the LDS planes.  Loads read clamped
// addresses inside the image; values outside it are replaced by 0, as in
// stage_tile.
template <class C>
struct TilePf {
  static constexpr int HALF = C::COLS / 2, NE = C::ROWS * HALF;
  static constexpr int NPT = (NE + C::NT - 1) / C::NT;   // pixel pairs per thread
  static constexpr int NPF = NPT < 16 ? NPT : 16;        // pairs prefetched
  const float* src;
  int H, W, r0, q0;
  float v[NPT][2];   // raw values (clamped reads), masked when stored
  // tile position of pair k; the opaque copy keeps the compiler from hoisting
  // every pair's address arithmetic out of the frame loop into registers
  __device__ void pos(int k, int& e, int& gy, int& gx) const {
    int kk = k * C::NT;
    __asm__ volatile("" : "+v"(kk));
    e = threadIdx.x + kk;
    const int row = e / HALF, cp = e - row * HALF;
    gy = r0 + row;
    gx = q0 + 2 * cp;
  }
  __device__ void load(int k) {
    int e, gy, gx;
    pos(k, e, gy, gx);
    const float* rp = src + (int64_t)min(max(gy, 0), H - 1) * W;
    v[k][0] = rp[min(max(gx, 0), W - 1)];
    v[k][1] = rp[min(max(gx + 1, 0), W - 1)];
  }
  __device__ void issue() {
#pragma unroll
    for (int k = 0; k < NPF; ++k) load(k);
  }
  __device__ void store(unsigned short (*sh)[C::ROWS * C::PITCH]) {
#pragma unroll
    for (int k = NPF; k < NPT; ++k) load(k);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      int e, gy, gx;
      pos(k, e, gy, gx);
      if (e < NE) {
        const bool iny = gy >= 0 && gy < H;
        const float v0 = (iny && gx >= 0 && gx < W) ? v[k][0] : 0.f;
        const float v1 = (iny && gx + 1 >= 0 && gx + 1 < W) ? v[k][1] : 0.f;
        const int o = (e / HALF) * C::PITCH + 2 * (e - (e / HALF) * HALF);
        unsigned short h0, l0, h1, l1;
        split_bf16(v0, h0, l0);
        split_bf16(v1, h1, l1);
        *reinterpret_cast<unsigned int*>(&sh[0][o]) = (unsigned int)h0 | ((unsigned int)h1 << 16);
        if constexpr (C::NA == 2)
          *reinterpret_cast<unsigned int*>(&sh[1][o]) = (unsigned int)l0 | ((unsigned int)l1 << 16);
      }
    }
  }
};

// Adjoint: sum over the frames of this group of F_t^T r_t; the r_t tile is
// staged per frame.  Epilogue: partial plane, or the fused update of Eq. (2).
template <class C>
__device__ inline void mfma_adj_body(const MfmaLaunch& a, const int tile, const int group) {
  constexpr int c = (C::KT - 1) / 2;
  __shared__ __align__(16) unsigned short sh[C::NA][C::ROWS * C::PITCH];
  __shared__ double red[2 * C::NW];
  __shared__ float redf[C::NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row_base = (w / C::WC) * 16 * C::BR, col_base = (w % C::WC) * 16 * C::BC;
  const int tiles_x = (a.W + C::TW - 1) / C::TW;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int k0 = ty * C::TH, l0 = tx * C::TW;
  const int64_t N = (int64_t)a.H * a.W;

  f32x4 acc[C::BR][C::BC];
#pragma unroll
  for (int b = 0; b < C::BR; ++b)
#pragma unroll
    for (int q = 0; q < C::BC; ++q) acc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const typename C::frag* tab = reinterpret_cast<const typename C::frag*>(a.tab);
  constexpr int64_t TSTRIDE = (int64_t)C::KTP * 4 * 64;   // fragments per frame
  __shared__ __align__(16) TBufDecl<C> tl;
  int step = 0;
  // unscaled encodings, register-held fragments, 8 waves: the next frame's tile
  // is prefetched during the current frame's classes (the 4-wave variant would
  // need twice the registers per thread)
  constexpr bool PF = C::PFT == 1 && !C::P::SCALED && C::NW == 8;
  std::conditional_t<PF, TilePf<C>, NoTilePf> pf;
  NoTilePf no_pf;
  if constexpr (PF) {
    pf.src = nullptr;
    pf.H = a.H;
    pf.W = a.W;
    pf.r0 = k0 - c;
    pf.q0 = l0 - c;
  }
  if constexpr (C::PFT == 2) issue_T<C>(tab + t0 * TSTRIDE, 0, (void*)&tl[0][0][0]);
  for (int t = t0; t < t1; ++t) {
    __syncthreads();
    int sr_t = 0;
    if (!PF || t == t0)
      sr_t = stage_tile<C::PREC, C::ROWS, C::COLS, C::PITCH, C::NT>(
          a.in + (int64_t)t * N, a.H, a.W, k0 - c, l0 - c, sh, redf);
    else if constexpr (PF)
      pf.store(sh);
    if constexpr (C::PFT == 2) frags_landed();
    else __syncthreads();
    const typename C::frag* tab_t = tab + t * TSTRIDE;
    const typename C::frag* tab_next = t + 1 < t1 ? tab_t + TSTRIDE : nullptr;
    if constexpr (C::P::SCALED) {
      // each frame has its own scales: sum it in its own accumulators, then
      // add it to the total unscaled (ldexp is exact)
      f32x4 accf[C::BR][C::BC];
#pragma unroll
      for (int b = 0; b < C::BR; ++b)
#pragma unroll
        for (int q = 0; q < C::BC; ++q) accf[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};
      if constexpr (C::PFT == 2)
        mfma_frame_lds<C>(sh, tab_t, tab_next, tl, step, row_base, col_base, accf);
      else
        mfma_frame<C>(sh, tab_t, row_base, col_base, accf, no_pf, false);
      const int unscale = -(sr_t + table_exponents<C>(a)[t]);
#pragma unroll
      for (int b = 0; b < C::BR; ++b)
#pragma unroll
        for (int q = 0; q < C::BC; ++q)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[b][q][v] += ldexpf(accf[b][q][v], unscale);
    } else {
      (void)sr_t;
      if constexpr (C::PFT == 2) {
        mfma_frame_lds<C>(sh, tab_t, tab_next, tl, step, row_base, col_base, acc);
      } else if constexpr (PF) {
        pf.src = a.in + (int64_t)(t + 1) * N;
        mfma_frame<C>(sh, tab_t, row_base, col_base, acc, pf, t + 1 < t1);
      } else {
        mfma_frame<C>(sh, tab_t, row_base, col_base, acc, no_pf, false);
      }
    }
  }

  double dsq = 0.0, xsq = 0.0;
  adjoint_epilogue<C::BR, C::BC>(acc, BlockPos{k0 + row_base, l0 + col_base, 1}, a.H, a.W,
                                 a.fused, a.x, a.B,
                                 a.fused ? nullptr : a.plane + (int64_t)group * N, dsq, xsq);
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
// Adjoint on binary16 r planes (FP16 split form): the forward has already
// written r_t scaled by 2^e16[t] as binary16, zero outside the frame, in planes
// laid out so that a tile's window (ROWS rows of COLS halves from plane row k0,
// column l0) is ROWS runs of 352 bytes starting on 16-byte boundaries.  The
// window is copied straight into LDS (global_load_lds_dwordx4, 1 KB per wave
// instruction, no registers, no conversion): the next frame's window goes into
// the second LDS buffer during the first classes of the current frame, one
// copy per wave and class, and may stay in flight for one more class, since a
// wave's loads complete in issue order and each class waits only until its
// own newest copy is the one outstanding.
// ---------------------------------------------------------------------------
constexpr int WAIT_VM0 = 0x0070;   // s_waitcnt vmcnt(0) lgkmcnt(0)
constexpr int WAIT_VM1 = 0x0071;   // s_waitcnt vmcnt(1) lgkmcnt(0)

template <class C>
struct Win16 {
  static constexpr int HALVES = C::ROWS * C::PITCH;      // one staged window
  static constexpr int BYTES = 2 * HALVES;
  static constexpr int ROW_BYTES = 2 * C::PITCH;
  static constexpr int NCH = (BYTES + 1023) / 1024;      // 1 KB copies per window
  static constexpr int CCL = (NCH + C::NW - 1) / C::NW;  // classes that carry copies
  static_assert(C::PITCH == C::COLS, "a window row is one contiguous run of its plane row");
  static_assert(ROW_BYTES % 16 == 0, "16-byte pieces never straddle window rows");
  // the last class of a frame carries no copy, so its wait completes the window
  static_assert(CCL < C::RLAST, "the copies fit in the classes of one frame");
};

// Copy chunk `ch` (bytes [1024 ch, 1024 ch + 1024) of the window) of the window
// at plane row k0, column l0 into LDS buffer dst; lanes past the window's end
// copy nothing.
template <class C>
__device__ inline void copy_window_chunk(const unsigned short* __restrict__ plane, int p16, int k0,
                                         int l0, int ch, unsigned short* dst) {
  using Wn = Win16<C>;
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

// One tap class of a frame whose window is in `sh`: read this class's Toeplitz
// fragments, start the copy of the next class's fragments, then this wave's
// copy of the next frame's window for this class (if any), issue the class's
// products, wait until at most the window copy is outstanding, meet at a
// barrier.  (Reading the fragments before the copies are issued keeps the
// compiler from waiting for the copies before the reads.)
template <class C, int NM>
__device__ inline void mfma_class_lds16(int r, const unsigned short (*sh)[C::ROWS * C::PITCH],
                                        const typename C::frag* __restrict__ tab_t,
                                        const typename C::frag* __restrict__ tab_next,
                                        TBuf<C>& tl, int& step, int row_base, int col_base,
                                        f32x4 (&acc)[C::BR][C::BC],
                                        const unsigned short* __restrict__ next_plane, int p16,
                                        int k0, int l0, unsigned short* next_buf) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cur = step & 1;
  typename C::frag Tc[C::MMAX][2][C::NB];
#pragma unroll
  for (int m = 0; m < C::MMAX; ++m)
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < C::NB; ++q) Tc[m][h][q] = tl[cur][(m * 2 + h) * C::NB + q][lane];
  if (r + 1 < C::RLAST) issue_T<C>(tab_t, r + 1, (void*)&tl[cur ^ 1][0][0]);
  else if (tab_next != nullptr) issue_T<C>(tab_next, 0, (void*)&tl[cur ^ 1][0][0]);
  const int ch = r * C::NW + w;
  const bool copied = next_plane != nullptr && r < Win16<C>::CCL && ch < Win16<C>::NCH;
  if (copied) copy_window_chunk<C>(next_plane, p16, k0, l0, ch, next_buf);
  mfma_class<C, NM>(r, sh, Tc, row_base, col_base, acc);
  if (copied) __builtin_amdgcn_s_waitcnt(WAIT_VM1);
  else __builtin_amdgcn_s_waitcnt(WAIT_VM0);
  __builtin_amdgcn_s_barrier();
  ++step;
}

template <class C>
__device__ inline void mfma_adj16_body(const MfmaLaunch& a, const int tile, const int group) {
  static_assert(C::PREC == EM_FP16_SPLIT && C::PFT == 2, "r16 planes feed the FP16 split form");
  using Wn = Win16<C>;
  __shared__ __align__(16) unsigned short rb[2][Wn::HALVES];
  __shared__ double red[2 * C::NW];
  __shared__ __align__(16) TBufDecl<C> tl;
  const int w = threadIdx.x >> 6;
  const int row_base = (w / C::WC) * 16 * C::BR, col_base = (w % C::WC) * 16 * C::BC;
  const int tiles_x = (a.W + C::TW - 1) / C::TW;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int k0 = ty * C::TH, l0 = tx * C::TW;
  const int64_t N = (int64_t)a.H * a.W;

  f32x4 acc[C::BR][C::BC];
#pragma unroll
  for (int b = 0; b < C::BR; ++b)
#pragma unroll
    for (int q = 0; q < C::BC; ++q) acc[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const typename C::frag* tab = reinterpret_cast<const typename C::frag*>(a.tab);
  constexpr int64_t TSTRIDE = (int64_t)C::KTP * 4 * 64;
  const int* e_tab = table_exponents<C>(a);
  int step = 0;
  // first frame: its window and its first class's fragments, all waves
  issue_T<C>(tab + t0 * TSTRIDE, 0, (void*)&tl[0][0][0]);
  for (int ch = w; ch < Wn::NCH; ch += C::NW)
    copy_window_chunk<C>(a.r16 + (int64_t)t0 * a.s16, a.p16, k0, l0, ch, &rb[0][0]);
  __builtin_amdgcn_s_waitcnt(WAIT_VM0);
  __builtin_amdgcn_s_barrier();
  for (int t = t0; t < t1; ++t) {
    const int buf = (t - t0) & 1;
    const unsigned short(*sh)[C::ROWS * C::PITCH] =
        reinterpret_cast<const unsigned short(*)[C::ROWS * C::PITCH]>(&rb[buf][0]);
    const bool more = t + 1 < t1;
    const unsigned short* next_plane = more ? a.r16 + (int64_t)(t + 1) * a.s16 : nullptr;
    const typename C::frag* tab_t = tab + t * TSTRIDE;
    const typename C::frag* tab_next = more ? tab_t + TSTRIDE : nullptr;
    f32x4 accf[C::BR][C::BC];
#pragma unroll
    for (int b = 0; b < C::BR; ++b)
#pragma unroll
      for (int q = 0; q < C::BC; ++q) accf[b][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    int r = 0;
#pragma unroll 1
    for (; r < C::RFULL; ++r)
      mfma_class_lds16<C, C::MMAX>(r, sh, tab_t, tab_next, tl, step, row_base, col_base, accf,
                                   next_plane, a.p16, k0, l0, &rb[buf ^ 1][0]);
    if constexpr (C::MMAX > 1) {
#pragma unroll 1
      for (; r < C::RLAST; ++r)
        mfma_class_lds16<C, C::MMAX - 1>(r, sh, tab_t, tab_next, tl, step, row_base, col_base,
                                         accf, next_plane, a.p16, k0, l0, &rb[buf ^ 1][0]);
    }
    // each frame has its own scales: add it to the total unscaled (exact)
    const int unscale = -(a.e16[t] + e_tab[t]);
#pragma unroll
    for (int b = 0; b < C::BR; ++b)
#pragma unroll
      for (int q = 0; q < C::BC; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[b][q][v] += ldexpf(accf[b][q][v], unscale);
  }

  double dsq = 0.0, xsq = 0.0;
  adjoint_epilogue<C::BR, C::BC>(acc, BlockPos{k0 + row_base, l0 + col_base, 1}, a.H, a.W,
                                 a.fused, a.x, a.B,
                                 a.fused ? nullptr : a.plane + (int64_t)group * N, dsq, xsq);
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

// Entry points: one job (grid = tiles x frame groups) or a batch of jobs
// (persistent workgroups striding over (job, tile, frame group) work items).
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_fwd_kernel(MfmaLaunch a) {
  mfma_fwd_body<C>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_fwd_t_kernel(MfmaLaunch a) {
  mfma_fwd_body<C, true>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_adj_kernel(MfmaLaunch a) {
  mfma_adj_body<C>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_fwd16_kernel(MfmaLaunch a) {
  mfma_fwd_body<C, false, true>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_adj16_kernel(MfmaLaunch a) {
  mfma_adj16_body<C>(a, blockIdx.x, blockIdx.y);
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_fwd_batched(const MfmaLaunch* __restrict__ descs,
                                                          const int4* __restrict__ items,
                                                          int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const int4 w = items[i];
    const MfmaLaunch d = descs[w.x];
    mfma_fwd_body<C>(d, w.y, w.z);
    __syncthreads();
  }
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_fwd_t_batched(const MfmaLaunch* __restrict__ descs,
                                                            const int4* __restrict__ items,
                                                            int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const int4 w = items[i];
    const MfmaLaunch d = descs[w.x];
    mfma_fwd_body<C, true>(d, w.y, w.z);
    __syncthreads();
  }
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_adj_batched(const MfmaLaunch* __restrict__ descs,
                                                          const int4* __restrict__ items,
                                                          int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const int4 w = items[i];
    const MfmaLaunch d = descs[w.x];
    mfma_adj_body<C>(d, w.y, w.z);
    __syncthreads();
  }
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_fwd16_batched(const MfmaLaunch* __restrict__ descs,
                                                            const int4* __restrict__ items,
                                                            int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const int4 w = items[i];
    const MfmaLaunch d = descs[w.x];
    mfma_fwd_body<C, false, true>(d, w.y, w.z);
    __syncthreads();
  }
}
template <class C>
__global__ __launch_bounds__(C::NT) void mfma_adj16_batched(const MfmaLaunch* __restrict__ descs,
                                                            const int4* __restrict__ items,
                                                            int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const int4 w = items[i];
    const MfmaLaunch d = descs[w.x];
    mfma_adj16_body<C>(d, w.y, w.z);
    __syncthreads();
  }
}

// Toeplitz fragment tables, one block per (frame, kernel row a): entry
// [t][a][h][s][lane] holds the 8 16-bit values U_a[32h + 8(lane/16) + e][lane%16],
// e = 0..7, of part s (0 = hi, 1 = lo) of g = flip(f) (dir 0, forward) or
// g = f (dir 1, adjoint), f zero-padded from K to KT.  Scaled encodings
// multiply g by 2^e_t (e_t = f16_scale_exp of max |f_t|) and store e_t as the
// t-th of n ints after the fragments of all n frames.
template <int PREC>
__global__ __launch_bounds__(256) void mfma_table_kernel(const float* psf, int n, int K, int KT,
                                                         int KTP, int dir, unsigned short* tab) {
  __shared__ float redf[4];
  const int t = blockIdx.x, a = blockIdx.y;   // a in [0, KTP); rows a >= KT are zero
  const int off = (KT - K) / 2;
  const float* f = psf + (int64_t)t * K * K;
  int ex = 0;
  if constexpr (Prec<PREC>::SCALED) {
    float mx = 0.f;
    for (int i = threadIdx.x; i < K * K; i += 256) mx = fmaxf(mx, fabsf(f[i]));
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) redf[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmaxf(fmaxf(redf[0], redf[1]), fmaxf(redf[2], redf[3]));
    ex = f16_scale_exp(mx);
    if (a == 0 && threadIdx.x == 0)
      reinterpret_cast<int*>(tab + (size_t)n * KTP * 4 * 64 * 8)[t] = ex;
  }
  const int idx = threadIdx.x;          // (h, s, lane) = 2 x 2 x 64
  const int lane = idx & 63, s = (idx >> 6) & 1, h = idx >> 7;
  const int j = lane & 15, gq = lane >> 4;
  unsigned short* dst = tab + ((((int64_t)t * KTP + a) * 2 + h) * 2 + s) * 64 * 8 + lane * 8;
  for (int e = 0; e < 8; ++e) {
    const int p = 32 * h + 8 * gq + e;
    const int b = p - j;                 // column of g
    float gv = 0.f;
    if (a < KT && b >= 0 && b < KT) {
      // g[a][b]: forward uses the 180-degree flip of f
      const int fa = dir == 0 ? KT - 1 - a : a;
      const int fb = dir == 0 ? KT - 1 - b : b;
      const int ia = fa - off, ib = fb - off;
      if (ia >= 0 && ia < K && ib >= 0 && ib < K) gv = f[ia * K + ib];
    }
    dst[e] = table_part<PREC>(Prec<PREC>::SCALED ? ldexpf(gv, ex) : gv, s);
  }
}

int mfma_table_rows(int KT) { return 16 * ((KT + 15) / 16); }

hipError_t launch_mfma_tables(const Geometry& g, const float* psf, void* tab_fwd, void* tab_adj,
                              hipStream_t s) {
  if (g.sr == 2) return launch_mfma2_tables(g, psf, tab_fwd, tab_adj, s);
  const int KTP = mfma_table_rows(g.KT);
  dim3 grid(g.n, KTP);
  for (int dir = 0; dir < 2; ++dir) {
    unsigned short* t = static_cast<unsigned short*>(dir == 0 ? tab_fwd : tab_adj);
    if (g.precision == EM_FP16_SPLIT)
      hipLaunchKernelGGL(mfma_table_kernel<EM_FP16_SPLIT>, grid, dim3(256), 0, s, psf, g.n, g.K,
                         g.KT, KTP, dir, t);
    else
      hipLaunchKernelGGL(mfma_table_kernel<EM_BF16_SPLIT>, grid, dim3(256), 0, s, psf, g.n, g.K,
                         g.KT, KTP, dir, t);
  }
  return hipGetLastError();
}

int mfma_tile_h() { return MF_TILE; }
int mfma_tile_w() { return MF_TILE; }

size_t mfma_table_bytes(const Geometry& g, int dir) {
  if (g.sr == 2) return dir == 0 && uses_m2n(g) ? mfma2n_table_bytes(g.n) : mfma2_table_bytes(g.n, dir);
  // fragments, then one scale exponent per frame
  return (size_t)g.n * mfma_table_rows(g.KT) * 4 * 64 * 8 * sizeof(uint16_t) +
         (size_t)g.n * sizeof(int);
}
int mfma_variants() { return 3; }

namespace {
// variant v: 0 = 4 waves of 4x4 blocks; 1 = 8 waves of 4x2 blocks; 2 = 8 waves of 2x4 blocks
template <int KT, int PREC>
hipError_t launch_dir(int dir, int variant, dim3 grid, const MfmaLaunch& a, hipStream_t s) {
  // Toeplitz fragments: staged in LDS for the one-plane binary16 image (LDS
  // traffic is low there), register prefetch for the two-plane bf16 split
  constexpr int PFT = PREC == EM_FP16_SPLIT ? 2 : 1;
  using C0 = MfCfg<KT, PREC, 4, 4, 2, 2, 1, PFT>;
  using C1 = MfCfg<KT, PREC, 4, 2, 2, 4, 0, PFT>;
  using C2 = MfCfg<KT, PREC, 2, 4, 4, 2, 0, PFT>;
  static_assert(C0::TH == MF_TILE && C0::TW == MF_TILE, "tile");
  static_assert(C1::TH == MF_TILE && C1::TW == MF_TILE, "tile");
  static_assert(C2::TH == MF_TILE && C2::TW == MF_TILE, "tile");
  if constexpr (PREC == EM_FP16_SPLIT) {
    if (a.r16 != nullptr && dir == 0) {
      // the 4x2-block forward on binary16 r planes loads the next fragment row
      // of the image before the products of the current one (4% faster there)
      using C1A = MfCfg<KT, PREC, 4, 2, 2, 4, 1, PFT>;
      if (variant == 1) hipLaunchKernelGGL(mfma_fwd16_kernel<C1A>, grid, dim3(C1A::NT), 0, s, a);
      else if (variant == 2) hipLaunchKernelGGL(mfma_fwd16_kernel<C2>, grid, dim3(C2::NT), 0, s, a);
      else hipLaunchKernelGGL(mfma_fwd16_kernel<C0>, grid, dim3(C0::NT), 0, s, a);
      return hipGetLastError();
    }
    if (a.r16 != nullptr) {
      if (variant == 1) hipLaunchKernelGGL(mfma_adj16_kernel<C1>, grid, dim3(C1::NT), 0, s, a);
      else if (variant == 2) hipLaunchKernelGGL(mfma_adj16_kernel<C2>, grid, dim3(C2::NT), 0, s, a);
      else hipLaunchKernelGGL(mfma_adj16_kernel<C0>, grid, dim3(C0::NT), 0, s, a);
      return hipGetLastError();
    }
  } else {
    if (a.r16 != nullptr) return hipErrorInvalidValue;
  }
  if constexpr (PREC == EM_BF16_SPLIT && KT == 43) {
    // the BF16 split iteration of a job whose PSFs pass the band check
    if (a.lo_band) {
      using B0 = MfCfg<KT, PREC, 4, 4, 2, 2, 1, PFT, 1>;
      using B1 = MfCfg<KT, PREC, 4, 2, 2, 4, 0, PFT, 1>;
      using B2 = MfCfg<KT, PREC, 2, 4, 4, 2, 0, PFT, 1>;
      if (dir == 0 && a.out_y != nullptr) {
        if (variant == 1) hipLaunchKernelGGL(mfma_fwd_t_kernel<B1>, grid, dim3(B1::NT), 0, s, a);
        else if (variant == 2) hipLaunchKernelGGL(mfma_fwd_t_kernel<B2>, grid, dim3(B2::NT), 0, s, a);
        else hipLaunchKernelGGL(mfma_fwd_t_kernel<B0>, grid, dim3(B0::NT), 0, s, a);
      } else if (dir == 0) {
        if (variant == 1) hipLaunchKernelGGL(mfma_fwd_kernel<B1>, grid, dim3(B1::NT), 0, s, a);
        else if (variant == 2) hipLaunchKernelGGL(mfma_fwd_kernel<B2>, grid, dim3(B2::NT), 0, s, a);
        else hipLaunchKernelGGL(mfma_fwd_kernel<B0>, grid, dim3(B0::NT), 0, s, a);
      } else {
        if (variant == 1) hipLaunchKernelGGL(mfma_adj_kernel<B1>, grid, dim3(B1::NT), 0, s, a);
        else if (variant == 2) hipLaunchKernelGGL(mfma_adj_kernel<B2>, grid, dim3(B2::NT), 0, s, a);
        else hipLaunchKernelGGL(mfma_adj_kernel<B0>, grid, dim3(B0::NT), 0, s, a);
      }
      return hipGetLastError();
    }
  }
  if (dir == 0 && a.out_y != nullptr) {
    if (variant == 1) hipLaunchKernelGGL(mfma_fwd_t_kernel<C1>, grid, dim3(C1::NT), 0, s, a);
    else if (variant == 2) hipLaunchKernelGGL(mfma_fwd_t_kernel<C2>, grid, dim3(C2::NT), 0, s, a);
    else hipLaunchKernelGGL(mfma_fwd_t_kernel<C0>, grid, dim3(C0::NT), 0, s, a);
  } else if (dir == 0) {
    if (variant == 1) hipLaunchKernelGGL(mfma_fwd_kernel<C1>, grid, dim3(C1::NT), 0, s, a);
    else if (variant == 2) hipLaunchKernelGGL(mfma_fwd_kernel<C2>, grid, dim3(C2::NT), 0, s, a);
    else hipLaunchKernelGGL(mfma_fwd_kernel<C0>, grid, dim3(C0::NT), 0, s, a);
  } else {
    if (variant == 1) hipLaunchKernelGGL(mfma_adj_kernel<C1>, grid, dim3(C1::NT), 0, s, a);
    else if (variant == 2) hipLaunchKernelGGL(mfma_adj_kernel<C2>, grid, dim3(C2::NT), 0, s, a);
    else hipLaunchKernelGGL(mfma_adj_kernel<C0>, grid, dim3(C0::NT), 0, s, a);
  }
  return hipGetLastError();
}
}  // namespace

namespace {
template <int KT, int PREC>
hipError_t launch_dir_batched(int dir, int variant, int grid, const MfmaLaunch* d, const int4* it,
                              int n, hipStream_t s, bool robust, bool r16) {
  // Toeplitz fragments: staged in LDS for the one-plane binary16 image (LDS
  // traffic is low there), register prefetch for the two-plane bf16 split
  constexpr int PFT = PREC == EM_FP16_SPLIT ? 2 : 1;
  using C0 = MfCfg<KT, PREC, 4, 4, 2, 2, 1, PFT>;
  using C1 = MfCfg<KT, PREC, 4, 2, 2, 4, 0, PFT>;
  using C2 = MfCfg<KT, PREC, 2, 4, 4, 2, 0, PFT>;
  if constexpr (PREC == EM_FP16_SPLIT) {
    if (r16 && dir == 0) {
      using C1A = MfCfg<KT, PREC, 4, 2, 2, 4, 1, PFT>;   // as in launch_dir
      if (variant == 1) hipLaunchKernelGGL(mfma_fwd16_batched<C1A>, dim3(grid), dim3(C1A::NT), 0, s, d, it, n);
      else if (variant == 2) hipLaunchKernelGGL(mfma_fwd16_batched<C2>, dim3(grid), dim3(C2::NT), 0, s, d, it, n);
      else hipLaunchKernelGGL(mfma_fwd16_batched<C0>, dim3(grid), dim3(C0::NT), 0, s, d, it, n);
      return hipGetLastError();
    }
    if (r16) {
      if (variant == 1) hipLaunchKernelGGL(mfma_adj16_batched<C1>, dim3(grid), dim3(C1::NT), 0, s, d, it, n);
      else if (variant == 2) hipLaunchKernelGGL(mfma_adj16_batched<C2>, dim3(grid), dim3(C2::NT), 0, s, d, it, n);
      else hipLaunchKernelGGL(mfma_adj16_batched<C0>, dim3(grid), dim3(C0::NT), 0, s, d, it, n);
      return hipGetLastError();
    }
  } else {
    if (r16) return hipErrorInvalidValue;
  }
  if (dir == 0 && robust) {
    if (variant == 1) hipLaunchKernelGGL(mfma_fwd_t_batched<C1>, dim3(grid), dim3(C1::NT), 0, s, d, it, n);
    else if (variant == 2) hipLaunchKernelGGL(mfma_fwd_t_batched<C2>, dim3(grid), dim3(C2::NT), 0, s, d, it, n);
    else hipLaunchKernelGGL(mfma_fwd_t_batched<C0>, dim3(grid), dim3(C0::NT), 0, s, d, it, n);
  } else if (dir == 0) {
    if (variant == 1) hipLaunchKernelGGL(mfma_fwd_batched<C1>, dim3(grid), dim3(C1::NT), 0, s, d, it, n);
    else if (variant == 2) hipLaunchKernelGGL(mfma_fwd_batched<C2>, dim3(grid), dim3(C2::NT), 0, s, d, it, n);
    else hipLaunchKernelGGL(mfma_fwd_batched<C0>, dim3(grid), dim3(C0::NT), 0, s, d, it, n);
  } else {
    if (variant == 1) hipLaunchKernelGGL(mfma_adj_batched<C1>, dim3(grid), dim3(C1::NT), 0, s, d, it, n);
    else if (variant == 2) hipLaunchKernelGGL(mfma_adj_batched<C2>, dim3(grid), dim3(C2::NT), 0, s, d, it, n);
    else hipLaunchKernelGGL(mfma_adj_batched<C0>, dim3(grid), dim3(C0::NT), 0, s, d, it, n);
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_mfma_batched(int KT, int precision, int dir, int variant, const MfmaLaunch* descs,
                               const int4* items, int n_items, int grid, hipStream_t s,
                               bool robust, bool r16) {
  if (n_items <= 0) return hipSuccess;
#define EM_MF_DISPATCH(KTV)                                                                  \
  switch (precision) {                                                                       \
    case EM_BF16_SPLIT:                                                                      \
      return launch_dir_batched<KTV, EM_BF16_SPLIT>(dir, variant, grid, descs, items, n_items, s, robust, r16); \
    case EM_FP16_SPLIT:                                                                      \
      return launch_dir_batched<KTV, EM_FP16_SPLIT>(dir, variant, grid, descs, items, n_items, s, robust, r16); \
    case EM_BF16:                                                                            \
      return launch_dir_batched<KTV, EM_BF16>(dir, variant, grid, descs, items, n_items, s, robust, r16); \
    default:                                                                                 \
      return hipErrorInvalidValue;                                                           \
  }
  if (KT == KT_LARGE) { EM_MF_DISPATCH(KT_LARGE) }
  EM_MF_DISPATCH(KT_SMALL)
#undef EM_MF_DISPATCH
}

bool mfma_desc_ok(const Geometry& g, int dir, int tiles, int groups, const MfmaLaunch& a) {
  // r16 planes: the plane geometry the set-up laid out, and the stride between frames
  if (a.r16 != nullptr &&
      (!uses_r16(g) || a.e16 == nullptr || a.p16 != r16_pitch(g) ||
       a.s16 != (int64_t)r16_rows(g) * r16_pitch(g) || a.out_y != nullptr || a.out != nullptr ||
       (dir == 1 && a.in != nullptr)))
    return false;
  if (g.sr == 2) return mfma2_desc_ok(g, dir, tiles, groups, a);
  return a.H == g.Hl && a.W == g.Wl &&
         launch_grid_ok(tiles, groups, a.ntiles, a.n, a.fpg, a.H, a.W, MF_TILE, MF_TILE);
}

int r16_pitch(const Geometry& g) {
  if (g.sr == 2) {
    // the FP16 split sr = 2 adjoint's windows: 176 halves from frame column L0/2
    const int tw = mfma2_adj_tile_w(EM_FP16_SPLIT);
    return tw / 2 * ((g.Wl + tw - 1) / tw) + 48;
  }
  return MF_TILE * ((g.Wl + MF_TILE - 1) / MF_TILE) + 48;
}
int r16_rows(const Geometry& g) {
  if (g.sr == 2) {
    // 96 frame rows from frame row K0/2
    const int th = mfma2_adj_tile_h(EM_FP16_SPLIT);
    return th / 2 * ((g.Hl + th - 1) / th) + 32;
  }
  return MF_TILE * ((g.Hl + MF_TILE - 1) / MF_TILE) + g.KT - 1;
}
int r16_off(const Geometry& g) { return g.sr == 2 ? 11 : (g.KT - 1) / 2; }

// Per frame (one block each): counts in *flag the frames whose PSF keeps more
// than 1/16 of its mass on the kernel rows outside the lo band (rows farther
// than 10 from the centre of the K-row stamp padded to 43).
__global__ __launch_bounds__(256) void lo_band_check_kernel(const float* psf, int K, int* flag) {
  __shared__ double red[2][4];
  const int t = blockIdx.x, off = (43 - K) / 2;
  const float* f = psf + (int64_t)t * K * K;
  double all = 0.0, outside = 0.0;
  for (int i = threadIdx.x; i < K * K; i += 256) {
    const double v = (double)f[i];
    const int a = i / K + off;
    all += v;
    if (a < 11 || a > 31) outside += v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    all += __shfl_xor(all, o, 64);
    outside += __shfl_xor(outside, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = all;
    red[1][threadIdx.x >> 6] = outside;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double A = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double O = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    if (!(16.0 * O <= A)) atomicAdd(flag, 1);
  }
}

hipError_t launch_lo_band_check(const Geometry& g, const float* psf, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(lo_band_check_kernel, dim3(g.n), dim3(256), 0, s, psf, g.K, flag);
  return hipGetLastError();
}

// Zero the r16 planes (16 bytes per thread).
__global__ __launch_bounds__(256) void r16_clear_kernel(uint4* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Per frame (one block each): the largest weight u_t and the sum of the absolute
// taps the forward applies (f_t, or for sr = 2 the 2x2 box-extended kernel,
// whose sum is fscale = 4 times that of f_t).
__global__ __launch_bounds__(1024) void r16_frame_stats_kernel(const float* u, int64_t Nf,
                                                               const float* psf, int K,
                                                               float fscale, float* umax,
                                                               float* fsum) {
  __shared__ float redm[16];
  __shared__ double reds[16];
  const int t = blockIdx.x;
  const float* ut = u + (int64_t)t * Nf;
  float m = 0.f;
  for (int64_t i = threadIdx.x; i < Nf; i += 1024) m = fmaxf(m, ut[i]);
  double sf = 0.0;
  for (int i = threadIdx.x; i < K * K; i += 1024) sf += fabs((double)psf[(int64_t)t * K * K + i]);
  m = wave_max(m);
  for (int off = 32; off > 0; off >>= 1) sf += __shfl_xor(sf, off, 64);
  if ((threadIdx.x & 63) == 0) {
    redm[threadIdx.x >> 6] = m;
    reds[threadIdx.x >> 6] = sf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float mm = 0.f;
    double ss = 0.0;
    for (int i = 0; i < 16; ++i) {
      mm = fmaxf(mm, redm[i]);
      ss += reds[i];
    }
    umax[t] = mm;
    fsum[t] = (float)(ss * fscale);
  }
}

// Block maxima of x (R16_XBLOCKS blocks, grid-stride).
// Largest |x[i]| over this thread's share of a grid-stride pass: 16-byte loads,
// four in flight per thread, when x is 16-byte aligned.
__device__ inline float abs_max_share(const float* __restrict__ x, int64_t Nl) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float m = 0.f;
  int64_t done = 0;
  if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const int64_t n4 = Nl >> 2;
#pragma unroll 4
    for (int64_t i = tid; i < n4; i += stride) {
      const float4 v = x4[i];
      m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    done = n4 << 2;
  }
  for (int64_t i = done + tid; i < Nl; i += stride) m = fmaxf(m, fabsf(x[i]));
  return m;
}

__global__ __launch_bounds__(256) void r16_xmax_kernel(const float* x, int64_t Nl, float* part) {
  __shared__ float red[4];
  float m = abs_max_share(x, Nl);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// e16[t]: the power of two that maps the bound 2 max u_t (sum |f_t|) max |x| of
// |u_t F_t x| into [2^14, 2^15) (|F_t x| <= sum |f_t| max |x|; the factor 2
// covers the rounding of the matrix-core products), so no
// scaled value overflows binary16 and values down to 2^-29 of the bound keep
// 11 significant bits.
__global__ __launch_bounds__(256) void r16_scale_kernel(const float* part, int nb,
                                                        const float* umax, const float* fsum,
                                                        int n, int* e16) {
  __shared__ float red[4];
  float m = 0.f;
  for (int i = threadIdx.x; i < nb; i += 256) m = fmaxf(m, part[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  const float xm = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  for (int t = threadIdx.x; t < n; t += 256) e16[t] = f16_scale_exp(2.f * umax[t] * fsum[t] * xm);
}

// Several jobs at once (serving): job j = blockIdx.y / blockIdx.x.
__global__ __launch_bounds__(256) void r16_xmax_batched_kernel(const R16Job* jobs) {
  __shared__ float red[4];
  const R16Job j = jobs[blockIdx.y];
  float m = abs_max_share(j.x, j.Nl);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) j.xpart[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void r16_scale_batched_kernel(const R16Job* jobs) {
  __shared__ float red[4];
  const R16Job j = jobs[blockIdx.x];
  float m = 0.f;
  for (int i = threadIdx.x; i < R16_XBLOCKS; i += 256) m = fmaxf(m, j.xpart[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  const float xm = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  for (int t = threadIdx.x; t < j.n; t += 256) j.e16[t] = f16_scale_exp(2.f * j.umax[t] * j.fsum[t] * xm);
}

hipError_t launch_r16_scale_batched(const R16Job* jobs, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(r16_xmax_batched_kernel, dim3(R16_XBLOCKS, n_jobs), dim3(256), 0, s, jobs);
  hipLaunchKernelGGL(r16_scale_batched_kernel, dim3(n_jobs), dim3(256), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_r16_setup(const Geometry& g, const float* u, const float* psf,
                            unsigned short* r16, float* umax, float* fsum, hipStream_t s) {
  const int64_t halves = (int64_t)g.n * r16_rows(g) * r16_pitch(g);   // multiple of 8
  const int64_t n16 = halves / 8;
  const int blocks = (int)std::min<int64_t>(8192, (n16 + 255) / 256);
  hipLaunchKernelGGL(r16_clear_kernel, dim3(std::max(blocks, 1)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(r16), n16);
  hipLaunchKernelGGL(r16_frame_stats_kernel, dim3(g.n), dim3(1024), 0, s, u, g.Nf, psf, g.K,
                     g.sr == 2 ? 4.f : 1.f, umax, fsum);
  return hipGetLastError();
}

hipError_t launch_r16_scale(const Geometry& g, const float* x, float* xpart, const float* umax,
                            const float* fsum, int* e16, hipStream_t s) {
  hipLaunchKernelGGL(r16_xmax_kernel, dim3(R16_XBLOCKS), dim3(256), 0, s, x, g.Nl, xpart);
  hipLaunchKernelGGL(r16_scale_kernel, dim3(1), dim3(256), 0, s, xpart, R16_XBLOCKS, umax, fsum,
                     g.n, e16);
  return hipGetLastError();
}

hipError_t launch_mfma(const Geometry& g, int dir, int variant, int tiles, int groups,
                       const MfmaLaunch& a, hipStream_t s) {
  if (g.sr == 2) return launch_mfma2(g, dir, variant, tiles, groups, a, s);
  if (!mfma_desc_ok(g, dir, tiles, groups, a)) return hipErrorInvalidValue;
  dim3 grid(tiles, groups);
#define EM_MF_DISPATCH(KTV)                                                  \
  switch (g.precision) {                                                     \
    case EM_BF16_SPLIT: return launch_dir<KTV, EM_BF16_SPLIT>(dir, variant, grid, a, s); \
    case EM_FP16_SPLIT: return launch_dir<KTV, EM_FP16_SPLIT>(dir, variant, grid, a, s); \
    case EM_BF16: return launch_dir<KTV, EM_BF16>(dir, variant, grid, a, s);             \
    default: return hipErrorInvalidValue;                                    \
  }
  if (g.KT == KT_LARGE) { EM_MF_DISPATCH(KT_LARGE) }
  EM_MF_DISPATCH(KT_SMALL)
#undef EM_MF_DISPATCH
}

}  // namespace em
