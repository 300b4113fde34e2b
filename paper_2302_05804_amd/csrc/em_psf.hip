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
// Layout: one workgroup of PSF_NT threads per frame; A, A^T, f, rho, T, U and
// two buffers of h (read one, write the other: one barrier per product) in
// LDS, every row padded to a multiple of 4 floats so that the right operand of
// each product is read 16 bytes at a time.  Each thread owns up to PSF_TPT
// 1 x 4 strips of h and keeps their Adam moments in registers for the whole
// run.  Arithmetic is binary32 except the schedule scalars and the final
// objective (binary64).
#include <hip/hip_runtime.h>
#include <math.h>

#include "em_device.h"
#include "em_internal.h"

namespace em {
namespace {

constexpr int PSF_NT = 512;
constexpr int PSF_TPT = (PSF_K_MAX * ((PSF_K_MAX + 3) / 4) + PSF_NT - 1) / PSF_NT;

__host__ __device__ constexpr int pad4(int k) { return (k + 3) & ~3; }

struct PsfLds {
  float *A, *At, *F, *R, *T, *U, *H0, *H1;
  double* red;
};

__host__ __device__ inline size_t psf_lds_floats(int kf, int kh) {
  const int pf = pad4(kf), ph = pad4(kh);
  return (size_t)kf * ph * 2 + (size_t)kh * pf * 2 + (size_t)kf * pf * 2 + (size_t)kh * ph * 2;
}

// out[r][c..c+3] = sum_{k < K} L[r][k] R[k][c..c+3]
__device__ inline float4 row_times(const float* L, int ldl, const float* R, int ldr, int r, int c,
                                   int K) {
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const float* lp = L + r * ldl;
  const float* rp = R + c;
#pragma unroll 4
  for (int k = 0; k < K; ++k) {
    const float l = lp[k];
    const float4 b = *reinterpret_cast<const float4*>(rp + k * ldr);
    acc.x = fmaf(l, b.x, acc.x);
    acc.y = fmaf(l, b.y, acc.y);
    acc.z = fmaf(l, b.z, acc.z);
    acc.w = fmaf(l, b.w, acc.w);
  }
  return acc;
}

// T = h A^T (kh x kf), then rho = A T - f (kf x kf); pads of T and rho are 0.
__device__ inline void psf_residual(const PsfLds& s, const float* H, int kf, int kh) {
  const int pf = pad4(kf), ph = pad4(kh);
  for (int q = threadIdx.x; q < kh * (pf / 4); q += PSF_NT) {
    const int a = q / (pf / 4), c = (q % (pf / 4)) * 4;
    *reinterpret_cast<float4*>(s.T + a * pf + c) = row_times(H, ph, s.At, pf, a, c, kh);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kf * (pf / 4); q += PSF_NT) {
    const int I = q / (pf / 4), c = (q % (pf / 4)) * 4;
    float4 m = row_times(s.A, ph, s.T, pf, I, c, kh);
    const float4 fv = *reinterpret_cast<const float4*>(s.F + I * pf + c);
    m.x -= fv.x;
    m.y -= fv.y;
    m.z -= fv.z;
    m.w -= fv.w;
    *reinterpret_cast<float4*>(s.R + I * pf + c) = m;
  }
  __syncthreads();
}

__device__ inline float h_at(const float* H, int ph, int kh, int a, int b) {
  return (a >= 0 && a < kh && b >= 0 && b < kh) ? H[a * ph + b] : 0.f;
}

__global__ __launch_bounds__(PSF_NT) void psf_fit_kernel(PsfParams P, const float* __restrict__ f,
                                                        const float* __restrict__ h0,
                                                        float* __restrict__ hout,
                                                        double* __restrict__ objective) {
  extern __shared__ float4 psf_smem4[];
  float* sm = reinterpret_cast<float*>(psf_smem4);
  const int kf = P.kf, kh = P.kh, D = P.D;
  const int pf = pad4(kf), ph = pad4(kh);
  const int t = blockIdx.x, tid = threadIdx.x;
  PsfLds s;
  s.A = sm;
  s.At = s.A + kf * ph;
  s.F = s.At + kh * pf;
  s.R = s.F + kf * pf;
  s.T = s.R + kf * pf;
  s.U = s.T + kh * pf;
  s.H0 = s.U + kf * ph;
  s.H1 = s.H0 + kh * ph;
  s.red = reinterpret_cast<double*>(s.H1 + kh * ph);
  const int nfl = (int)psf_lds_floats(kf, kh);
  for (int i = tid; i < nfl; i += PSF_NT) sm[i] = 0.f;
  __syncthreads();

  // A and A^T from the 1-D Gaussian (binary64, rounded once)
  const int ch = (kh - 1) / 2, anchor = D * ((kf - 1) / 2);
  const double sg = (double)P.sigma;
  const int rg = sg > 0.0 ? (int)ceil(4.0 * sg) : 0;
  double Z = 0.0;
  for (int d = -rg; d <= rg; ++d) Z += sg > 0.0 ? exp(-(double)(d * d) / (2.0 * sg * sg)) : 1.0;
  for (int q = tid; q < kf * kh; q += PSF_NT) {
    const int I = q / kh, a = q % kh;
    double v = 0.0;
    for (int p = D * I; p < D * I + D; ++p) {
      const int d = p - anchor - (a - ch);
      if (d >= -rg && d <= rg) v += sg > 0.0 ? exp(-(double)(d * d) / (2.0 * sg * sg)) : 1.0;
    }
    s.A[I * ph + a] = (float)(v / Z);
    s.At[a * pf + I] = (float)(v / Z);
  }
  // f, its maximum, and the start h
  const float* ft = f + (size_t)t * kf * kf;
  float fmax = 0.f;
  for (int q = tid; q < kf * kf; q += PSF_NT) {
    const float v = ft[q];
    s.F[(q / kf) * pf + q % kf] = v;
    fmax = fmaxf(fmax, v);
  }
  for (int q = tid; q < kh * kh; q += PSF_NT) {
    const int a = q / kh, b = q % kh;
    float v;
    if (h0) {
      v = h0[(size_t)t * kh * kh + q];
    } else {
      const int p = a - ch + anchor, r = b - ch + anchor;
      v = 0.f;
      if (p >= 0 && p < D * kf && r >= 0 && r < D * kf)
        v = fmaxf(ft[(p / D) * kf + r / D] / (float)(D * D), 0.f);
    }
    s.H0[a * ph + b] = v;
  }
  // block maximum of f (reduction through the doubles of s.red)
  {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) fmax = fmaxf(fmax, __shfl_xor(fmax, off, 64));
    if ((tid & 63) == 0) s.red[tid >> 6] = (double)fmax;
    __syncthreads();
    for (int w = 0; w < PSF_NT / 64; ++w) fmax = fmaxf(fmax, (float)s.red[w]);
    __syncthreads();
  }

  // Adam state of the owned strips
  float m1[PSF_TPT][4], m2[PSF_TPT][4];
#pragma unroll
  for (int j = 0; j < PSF_TPT; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) m1[j][e] = m2[j][e] = 0.f;

  const double lr0 = (double)P.lr * (double)fmax;
  const double ldec = P.S > 1 ? log((double)P.decay) / (double)(P.S - 1) : 0.0;
  const float b1 = P.b1, b2 = P.b2, eps = P.eps, lam2 = 2.f * P.lam;
  double b1k = 1.0, b2k = 1.0;
  float* Hc = s.H0;
  float* Hn = s.H1;
  for (int k = 1; k <= P.S; ++k) {
    psf_residual(s, Hc, kf, kh);
    // U = rho A (kf x kh)
    for (int q = tid; q < kf * (ph / 4); q += PSF_NT) {
      const int I = q / (ph / 4), c = (q % (ph / 4)) * 4;
      *reinterpret_cast<float4*>(s.U + I * ph + c) = row_times(s.R, pf, s.A, ph, I, c, kf);
    }
    __syncthreads();
    b1k *= (double)b1;
    b2k *= (double)b2;
    const float lrk = (float)(lr0 * exp(ldec * (double)(k - 1)));
    const float c1 = (float)(1.0 - b1k), c2 = (float)(1.0 - b2k);
#pragma unroll
    for (int j = 0; j < PSF_TPT; ++j) {
      const int q = tid + j * PSF_NT;
      if (q < kh * (ph / 4)) {
        const int a = q / (ph / 4), c = (q % (ph / 4)) * 4;
        const float4 gd = row_times(s.At, pf, s.U, ph, a, c, kf);
        const float gv[4] = {gd.x, gd.y, gd.z, gd.w};
        float hn[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int b = c + e;
          const float hv = h_at(Hc, ph, kh, a, b);
          const float nb = h_at(Hc, ph, kh, a - 1, b) + h_at(Hc, ph, kh, a + 1, b) +
                           h_at(Hc, ph, kh, a, b - 1) + h_at(Hc, ph, kh, a, b + 1);
          const float g = 2.f * gv[e] + lam2 * (4.f * hv - nb);
          m1[j][e] = b1 * m1[j][e] + (1.f - b1) * g;
          m2[j][e] = b2 * m2[j][e] + (1.f - b2) * g * g;
          const float step = lrk * (m1[j][e] / c1) / (sqrtf(m2[j][e] / c2) + eps);
          hn[e] = b < kh ? fmaxf(hv - step, 0.f) : 0.f;
        }
        *reinterpret_cast<float4*>(Hn + a * ph + c) = make_float4(hn[0], hn[1], hn[2], hn[3]);
      }
    }
    __syncthreads();
    float* tmp = Hc;
    Hc = Hn;
    Hn = tmp;
  }

  float* ht = hout + (size_t)t * kh * kh;
  for (int q = tid; q < kh * kh; q += PSF_NT) ht[q] = Hc[(q / kh) * ph + q % kh];
  if (objective) {
    psf_residual(s, Hc, kf, kh);
    double part = 0.0;
    for (int q = tid; q < kf * kf; q += PSF_NT) {
      const double r = (double)s.R[(q / kf) * pf + q % kf];
      part += r * r;
    }
    double pen = 0.0;
    for (int q = tid; q < (kh + 1) * kh; q += PSF_NT) {
      // pair (i, i+1) in column j and pair (j, j+1) in row j' = i (transposed)
      const int i = q / kh - 1, j = q % kh;
      const double dv = (double)h_at(Hc, ph, kh, i + 1, j) - (double)h_at(Hc, ph, kh, i, j);
      const double dh = (double)h_at(Hc, ph, kh, j, i + 1) - (double)h_at(Hc, ph, kh, j, i);
      pen += dv * dv + dh * dh;
    }
    const double tot = block_sum<PSF_NT>(part + (double)P.lam * pen, s.red);
    if (tid == 0) objective[t] = tot;
  }
}

}  // namespace

size_t psf_lds_bytes(int kf, int kh) {
  return psf_lds_floats(kf, kh) * sizeof(float) + (PSF_NT / 64) * sizeof(double);
}

hipError_t launch_psf_fit(const PsfParams& P, const float* f, const float* h0, float* h,
                          double* objective, hipStream_t s) {
  const size_t lds = psf_lds_bytes(P.kf, P.kh);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&psf_fit_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(psf_fit_kernel, dim3(P.n), dim3(PSF_NT), lds, s, P, f, h0, h, objective);
  return hipGetLastError();
}

}  // namespace em
