// em_psf.hip -- super-resolved PSFs of Eq. (4) (arXiv:2302.05804, Sec. 2) by
// projected Adam, every frame's fit in one workgroup.
//
// For a frame-grid PSF f (Kf x Kf) the fit seeks h >= 0 (Kh x Kh, fine grid)
// minimising |D(h * g) - f|^2 + lambda |grad h|^2.  g is an isotropic Gaussian,
// so D(h * g) on f's stamp factors as A h A^T with A a Kf x Kh matrix:
//     A[I][a] = sum_{p = D I}^{D I + D - 1} g1(p - anchor - (a - ch)),
// g1 the 1-D Gaussian (unit sum over |d| <= ceil(4 sigma)), anchor = D (Kf-1)/2
// the fine pixel that carries h's centre ch.  Rows of h*g that fall outside
// the D Kf fine stamp belong to no block I and drop out, as in the definition.
// One Adam step is then four small products that stay in LDS:
//     T = h A^T,  rho = A T - f,  U = rho A,  grad = 2 A^T U + 2 lambda L h,
// L the 5-point Laplacian of h extended by zeros (the derivative of the sum
// of squared forward differences), followed by Adam's moment update
// (Kingma & Ba, 2015, Algorithm 1), the step lr max(f) decay^((k-1)/(S-1))
// and the projection max(h, 0).
//
// Layout: one workgroup per frame; A, A^T, f, rho, T^T, U^T and two buffers of
// h (read one, write the other) in LDS, each padded with zeros to KP x KP
// (KP the multiple of 16 at or above Kf and Kh).  The products run on the
// matrix cores in binary32 (v_mfma_f32_16x16x4f32), one 16 x 16 output block
// per wave, so a workgroup has (KP/16)^2 waves; each lane reads 16-byte runs of
// its row of the left operand and of the transposed right operand, and the
// products that feed another one store their result transposed (T^T, U^T) so
// that the next product reads it the same way.  A lane keeps the Adam moments
// of the four pixels of its accumulator for the whole run.  One barrier
// follows each product.  Arithmetic is binary32 except the schedule scalars
// and the final objective (binary64).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "em_device.h"
#include "em_internal.h"

namespace em {
namespace {

typedef __attribute__((ext_vector_type(4))) float psf_f32x4;

// Every matrix is held padded to KP x KP (KP = 16, 32, 48 or 64, the multiple of
// 16 at or above Kf and Kh) with zeros outside its Kf / Kh extent, rows PP
// floats apart.  One wave per 16 x 16 output block.
template <int KP>
struct PsfShape {
  static constexpr int NB = KP / 16;          // output blocks per side
  static constexpr int NW = NB * NB;          // waves (one block each)
  static constexpr int NT = 64 * NW;
  static constexpr int KS = KP / 4;           // k values per lane group
  static constexpr int PP = KP + 4;           // row pitch (floats)
  static constexpr int MAT = KP * PP;         // floats per matrix
  static constexpr int NMAT = 8;              // A, At, F, R, Tt, Ut, H0, H1
};

// C block (bm, bn) of L * R with R given transposed (Rt[n][k]): lane i supplies
// L[16 bm + i%16][k] and Rt[16 bn + i%16][k] for the k values of its lane group
// g = i/16, k in [g KS, g KS + KS).  The matrix instruction sums its four lane
// groups, so every k is taken once.  Returns C[16 bm + 4 g + j][16 bn + i%16]
// in element j.
template <int KP>
__device__ inline psf_f32x4 psf_block(const float* L, const float* Rt, int bm, int bn) {
  using S = PsfShape<KP>;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const float* lp = L + (16 * bm + r) * S::PP + g * S::KS;
  const float* rp = Rt + (16 * bn + r) * S::PP + g * S::KS;
  // four independent accumulators, so that consecutive matrix instructions do
  // not wait for each other's results
  psf_f32x4 acc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[e] = psf_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int c = 0; c < S::KS; c += 4) {
    const float4 a4 = *reinterpret_cast<const float4*>(lp + c);
    const float4 b4 = *reinterpret_cast<const float4*>(rp + c);
    acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.x, b4.x, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.y, b4.y, acc[1], 0, 0, 0);
    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.z, b4.z, acc[2], 0, 0, 0);
    acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4.w, b4.w, acc[3], 0, 0, 0);
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Tt = (h A^T)^T, then R = A T - F (pads stay 0: A and F are 0 there).
template <int KP>
__device__ inline void psf_residual(const float* A, const float* H, const float* F, float* Tt,
                                    float* R, int bm, int bn) {
  using S = PsfShape<KP>;
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const psf_f32x4 t = psf_block<KP>(H, A, bm, bn);            // T[a][J], a = 16bm+4g+j
  *reinterpret_cast<psf_f32x4*>(Tt + (16 * bn + r) * S::PP + 16 * bm + 4 * g) = t;
  __syncthreads();
  const psf_f32x4 m = psf_block<KP>(A, Tt, bm, bn);           // M[I][J], I = 16bm+4g+j
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = (16 * bm + 4 * g + j) * S::PP + 16 * bn + r;
    R[o] = m[j] - F[o];
  }
  __syncthreads();
}

template <int KP>
__global__ __launch_bounds__(PsfShape<KP>::NT) void psf_fit_kernel(PsfParams P,
                                                                  const float* __restrict__ f,
                                                                  const float* __restrict__ h0,
                                                                  float* __restrict__ hout,
                                                                  double* __restrict__ objective) {
  using S = PsfShape<KP>;
  extern __shared__ float4 psf_smem4[];
  float* sm = reinterpret_cast<float*>(psf_smem4);
  float* A = sm;
  float* At = A + S::MAT;
  float* F = At + S::MAT;
  float* R = F + S::MAT;
  float* Tt = R + S::MAT;
  float* Ut = Tt + S::MAT;
  float* Hc = Ut + S::MAT;
  float* Hn = Hc + S::MAT;
  double* red = reinterpret_cast<double*>(Hn + S::MAT);
  const int kf = P.kf, kh = P.kh, D = P.D;
  const int t = blockIdx.x, tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
  const int bm = w / S::NB, bn = w % S::NB;
  for (int i = tid; i < S::NMAT * S::MAT; i += S::NT) sm[i] = 0.f;
  __syncthreads();

  // A[I][a] = sum over the D fine rows of coarse row I of g1(p - anchor - (a - ch)),
  // g1 the unit-sum 1-D Gaussian (binary64, rounded once); A^T beside it
  const int ch = (kh - 1) / 2, anchor = D * ((kf - 1) / 2);
  const double sg = (double)P.sigma;
  const int rg = sg > 0.0 ? (int)ceil(4.0 * sg) : 0;
  double Z = 0.0;
  for (int d = -rg; d <= rg; ++d) Z += sg > 0.0 ? exp(-(double)(d * d) / (2.0 * sg * sg)) : 1.0;
  for (int q = tid; q < kf * kh; q += S::NT) {
    const int I = q / kh, a = q % kh;
    double v = 0.0;
    for (int p = D * I; p < D * I + D; ++p) {
      const int d = p - anchor - (a - ch);
      if (d >= -rg && d <= rg) v += sg > 0.0 ? exp(-(double)(d * d) / (2.0 * sg * sg)) : 1.0;
    }
    A[I * S::PP + a] = (float)(v / Z);
    At[a * S::PP + I] = (float)(v / Z);
  }
  // f, its maximum, and the start h
  const float* ft = f + (size_t)t * kf * kf;
  float fmax = 0.f;
  for (int q = tid; q < kf * kf; q += S::NT) {
    const float v = ft[q];
    F[(q / kf) * S::PP + q % kf] = v;
    fmax = fmaxf(fmax, v);
  }
  for (int q = tid; q < kh * kh; q += S::NT) {
    const int a = q / kh, b = q % kh;
    float v;
    if (h0) {
      v = h0[(size_t)t * kh * kh + q];
    } else {
      const int p = a - ch + anchor, c2 = b - ch + anchor;
      v = 0.f;
      if (p >= 0 && p < D * kf && c2 >= 0 && c2 < D * kf)
        v = fmaxf(ft[(p / D) * kf + c2 / D] / (float)(D * D), 0.f);
    }
    Hc[a * S::PP + b] = v;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) fmax = fmaxf(fmax, __shfl_xor(fmax, off, 64));
  if (lane == 0) red[w] = (double)fmax;
  __syncthreads();
  for (int i = 0; i < S::NW; ++i) fmax = fmaxf(fmax, (float)red[i]);
  __syncthreads();

  // Adam state of the lane's four pixels (a = 16 bm + 4 g + j, b = 16 bn + r)
  float m1[4] = {0.f, 0.f, 0.f, 0.f}, m2[4] = {0.f, 0.f, 0.f, 0.f};
  // step k uses lr max(f) decay^((k-1)/(S-1)): a running product in binary64
  double lrk_d = (double)P.lr * (double)fmax;
  const double rdec = P.S > 1 ? exp(log((double)P.decay) / (double)(P.S - 1)) : 1.0;
  const float b1 = P.b1, b2 = P.b2, eps = P.eps, lam2 = 2.f * P.lam;
  const int b = 16 * bn + r;
  double b1k = 1.0, b2k = 1.0;
  for (int k = 1; k <= P.S; ++k) {
    psf_residual<KP>(A, Hc, F, Tt, R, bm, bn);
    // U = rho A, stored transposed (Ut[b][I])
    const psf_f32x4 u = psf_block<KP>(R, At, bm, bn);
    *reinterpret_cast<psf_f32x4*>(Ut + (16 * bn + r) * S::PP + 16 * bm + 4 * g) = u;
    __syncthreads();
    // gradient 2 A^T U + 2 lambda L h, Adam, projection
    const psf_f32x4 gd = psf_block<KP>(At, Ut, bm, bn);
    b1k *= (double)b1;
    b2k *= (double)b2;
    const float lrk = (float)lrk_d;
    lrk_d *= rdec;
    const float c1 = (float)(1.0 - b1k), c2 = (float)(1.0 - b2k);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = 16 * bm + 4 * g + j;
      float hn = 0.f;
      if (a < kh && b < kh) {
        const float hv = Hc[a * S::PP + b];
        const float nb = (a > 0 ? Hc[(a - 1) * S::PP + b] : 0.f) +
                         (a + 1 < kh ? Hc[(a + 1) * S::PP + b] : 0.f) +
                         (b > 0 ? Hc[a * S::PP + b - 1] : 0.f) +
                         (b + 1 < kh ? Hc[a * S::PP + b + 1] : 0.f);
        const float gr = 2.f * gd[j] + lam2 * (4.f * hv - nb);
        m1[j] = b1 * m1[j] + (1.f - b1) * gr;
        m2[j] = b2 * m2[j] + (1.f - b2) * gr * gr;
        const float step = lrk * (m1[j] / c1) / (sqrtf(m2[j] / c2) + eps);
        hn = fmaxf(hv - step, 0.f);
      }
      Hn[a * S::PP + b] = hn;
    }
    __syncthreads();
    float* tmp = Hc;
    Hc = Hn;
    Hn = tmp;
  }

  float* ht = hout + (size_t)t * kh * kh;
  for (int q = tid; q < kh * kh; q += S::NT) ht[q] = Hc[(q / kh) * S::PP + q % kh];
  if (objective) {
    psf_residual<KP>(A, Hc, F, Tt, R, bm, bn);
    double part = 0.0;
    for (int q = tid; q < kf * kf; q += S::NT) {
      const double rr = (double)R[(q / kf) * S::PP + q % kf];
      part += rr * rr;
    }
    double pen = 0.0;
    auto hat = [&](int i, int j) -> double {
      return (i >= 0 && i < kh && j >= 0 && j < kh) ? (double)Hc[i * S::PP + j] : 0.0;
    };
    for (int q = tid; q < (kh + 1) * kh; q += S::NT) {
      // pair (i, i+1) in column j, and pair (i, i+1) along row j
      const int i = q / kh - 1, j = q % kh;
      const double dv = hat(i + 1, j) - hat(i, j);
      const double dh = hat(j, i + 1) - hat(j, i);
      pen += dv * dv + dh * dh;
    }
    const double tot = block_sum<S::NT>(part + (double)P.lam * pen, red);
    if (tid == 0) objective[t] = tot;
  }
}

inline int psf_kp(int kf, int kh) { return 16 * ((std::max(kf, kh) + 15) / 16); }

template <int KP>
hipError_t launch_kp(const PsfParams& P, const float* f, const float* h0, float* h,
                     double* objective, hipStream_t s) {
  using S = PsfShape<KP>;
  const size_t lds = (size_t)S::NMAT * S::MAT * sizeof(float) + S::NW * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&psf_fit_kernel<KP>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(psf_fit_kernel<KP>, dim3(P.n), dim3(S::NT), lds, s, P, f, h0, h, objective);
  return hipGetLastError();
}

}  // namespace

size_t psf_lds_bytes(int kf, int kh) {
  const int kp = psf_kp(kf, kh);
  return (size_t)8 * kp * (kp + 4) * sizeof(float) + (size_t)(kp / 16) * (kp / 16) * sizeof(double);
}

hipError_t launch_psf_fit(const PsfParams& P, const float* f, const float* h0, float* h,
                          double* objective, hipStream_t s) {
  switch (psf_kp(P.kf, P.kh)) {
    case 16: return launch_kp<16>(P, f, h0, h, objective, s);
    case 32: return launch_kp<32>(P, f, h0, h, objective, s);
    case 48: return launch_kp<48>(P, f, h0, h, objective, s);
    case 64: return launch_kp<64>(P, f, h0, h, objective, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace em
