// em_elem.hip -- per-pixel and reduction kernels around the convolutions:
// weights u = 1/v and validation (text after Eq. (2) of arXiv:2302.05804),
// coefficient tables of F_t (Eq. (1) / Eq. (3)), the stand-alone update of
// Eq. (2) used when the adjoint is split over frame groups, and the FP64
// reductions (log-likelihood of Eq. (1), relative change, flat start).
// These are HBM-bound passes: grid-stride loops with coalesced accesses.
#include <math.h>

#include <algorithm>

#include "em_device.h"
#include "em_internal.h"

namespace em {

constexpr int EW_NT = 256;

// u = 1/v (0 where v = +inf), w = u * y (or y alone when raw_y; 0 where
// masked in both), FP64 partials of
// sum u y, sum u and sum_{u>0} ln(2 pi v); counts invalid pixels.
__global__ __launch_bounds__(EW_NT) void prep_kernel(PrepLaunch a) {
  __shared__ double red[3 * EW_NT / 64];
  double suy = 0.0, su = 0.0, sl = 0.0;
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * EW_NT;
  for (int64_t p = (int64_t)blockIdx.x * EW_NT + threadIdx.x; p < a.count; p += stride) {
    const float vv = a.v[p];
    const float yy = a.y[p];
    float uu = 0.f, ww = 0.f;
    if (isinf(vv) && vv > 0.f) {
      // masked pixel
    } else if (!(vv > 0.f) || !isfinite(vv) || !isfinite(yy)) {
      ++bad;
    } else {
      uu = 1.0f / vv;
      ww = a.raw_y ? yy : uu * yy;
      suy += (double)yy / (double)vv;
      su += 1.0 / (double)vv;
      sl += log(2.0 * M_PI * (double)vv);
    }
    a.u[p] = uu;
    a.w[p] = ww;
  }
  if (bad) atomicAdd(a.flags, bad);
  const double s0 = block_sum<EW_NT>(suy, red);
  __syncthreads();
  const double s1 = block_sum<EW_NT>(su, red + EW_NT / 64);
  __syncthreads();
  const double s2 = block_sum<EW_NT>(sl, red + 2 * EW_NT / 64);
  if (threadIdx.x == 0) {
    a.part[3 * blockIdx.x + 0] = s0;
    a.part[3 * blockIdx.x + 1] = s1;
    a.part[3 * blockIdx.x + 2] = s2;
  }
}

hipError_t launch_prep(const PrepLaunch& a, hipStream_t s) {
  hipLaunchKernelGGL(prep_kernel, dim3(a.blocks), dim3(EW_NT), 0, s, a);
  return hipGetLastError();
}

// Coefficient table of frame t (one block per frame), column-major with
// column pitch TAB_LD:
//   sr = 1: tab[b][a] = f_pad[a][b], f zero-padded from K to KT symmetrically;
//   sr = 2: tab[b'][a'] = sum_{p,q in {0,1}} f_pad[a'+p-1][b'+q-1]  (a',b' in [0,KT]),
//           the kernel of the 2x2 box sum of f * x read at stride 2 (Eq. (3)).
// Invalid taps (negative or not finite) are counted in flags[1].
__global__ __launch_bounds__(EW_NT) void psf_table_kernel(const float* psf, float* tab, int K,
                                                          int KT, int sr, int* flags) {
  const int t = blockIdx.x;
  const int off = (KT - K) / 2;
  const float* f = psf + (int64_t)t * K * K;
  const int KC = sr == 1 ? KT : KT + 1;
  float* tb = tab + (int64_t)t * KC * TAB_LD;
  int bad = 0;
  for (int e = threadIdx.x; e < K * K; e += EW_NT) {
    const float fv = f[e];
    if (!(fv >= 0.f) || !isfinite(fv)) ++bad;
  }
  if (bad) atomicAdd(flags + 1, bad);
  auto fp = [&](int a, int b) -> float {  // padded PSF, zero outside
    const int ia = a - off, ib = b - off;
    if (ia < 0 || ia >= K || ib < 0 || ib >= K) return 0.f;
    return f[ia * K + ib];
  };
  for (int e = threadIdx.x; e < KC * TAB_LD; e += EW_NT) {
    const int b = e / TAB_LD, a = e - b * TAB_LD;
    float val = 0.f;
    if (a < KC) {
      if (sr == 1) {
        val = fp(a, b);
      } else {
        val = (fp(a - 1, b - 1) + fp(a - 1, b)) + (fp(a, b - 1) + fp(a, b));
      }
    }
    tb[e] = val;
  }
}

hipError_t launch_psf_tables(const Geometry& g, const float* psf, float* tab, int* flags,
                             hipStream_t s) {
  hipLaunchKernelGGL(psf_table_kernel, dim3(g.n), dim3(EW_NT), 0, s, psf, tab, g.K, g.KT, g.sr,
                     flags);
  return hipGetLastError();
}

// Fixed-order FP64 sum of `count` values spaced `stride` apart, one block.
__device__ double ordered_sum(const double* p, int count, int stride, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += EW_NT) acc += p[(int64_t)i * stride];
  return block_sum<EW_NT>(acc, red);
}

__global__ __launch_bounds__(EW_NT) void finalize_prep_kernel(const double* part, int blocks,
                                                              double* sc, int sr) {
  __shared__ double red[EW_NT / 64];
  const double suy = ordered_sum(part + 0, blocks, 3, red);
  __syncthreads();
  const double su = ordered_sum(part + 1, blocks, 3, red);
  __syncthreads();
  const double sl = ordered_sum(part + 2, blocks, 3, red);
  if (threadIdx.x == 0) {
    sc[S_SUM_UY] = suy;
    sc[S_SUM_U] = su;
    sc[S_LCONST] = sl;
    double mu = su > 0.0 ? suy / su : 0.0;
    if (!(mu > 1e-3)) mu = 1e-3;
    sc[S_X0] = mu / (double)(sr * sr);
  }
}

hipError_t launch_finalize_prep(const double* part, int blocks, double* scalars, int sr,
                                hipStream_t s) {
  hipLaunchKernelGGL(finalize_prep_kernel, dim3(1), dim3(EW_NT), 0, s, part, blocks, scalars, sr);
  return hipGetLastError();
}

// x <- x0 (validated: finite and >= 0, else flags[2]) or the flat value.
__global__ __launch_bounds__(EW_NT) void init_x_kernel(const float* x0, float* x,
                                                       const double* sc, int64_t count,
                                                       int* flags) {
  const int64_t stride = (int64_t)gridDim.x * EW_NT;
  const float flat = (float)sc[S_X0];
  int bad = 0;
  for (int64_t p = (int64_t)blockIdx.x * EW_NT + threadIdx.x; p < count; p += stride) {
    float val = flat;
    if (x0 != nullptr) {
      val = x0[p];
      if (!(val >= 0.f) || !isfinite(val)) ++bad;
    }
    x[p] = val;
  }
  if (bad) atomicAdd(flags + 2, bad);
}

static int ew_blocks(int64_t count) {
  int64_t b = (count + EW_NT - 1) / EW_NT;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_init_x(const float* x0, float* x, const double* scalars, int64_t count,
                         int* flags, hipStream_t s) {
  hipLaunchKernelGGL(init_x_kernel, dim3(ew_blocks(count)), dim3(EW_NT), 0, s, x0, x, scalars,
                     count, flags);
  return hipGetLastError();
}

// Sum of G planes at pixel p in order g = 0..G-1; with per-plane weights w
// (the typeset weighting of Eq. (2): plane g is frame g's adjoint and w holds
// the frames' u on the same grid) each plane is multiplied by its weight first.
__device__ inline float plane_sum(const float* planes, const float* w, int G, int64_t Nl,
                                  int64_t p) {
  if (w == nullptr) {
    float acc = planes[p];
    for (int g = 1; g < G; ++g) acc += planes[(int64_t)g * Nl + p];
    return acc;
  }
  float acc = w[p] * planes[p];
  for (int g = 1; g < G; ++g) acc = fmaf(w[(int64_t)g * Nl + p], planes[(int64_t)g * Nl + p], acc);
  return acc;
}

__global__ __launch_bounds__(EW_NT) void sum_planes_kernel(const float* planes, const float* w,
                                                           int G, int64_t Nl, float* out) {
  const int64_t stride = (int64_t)gridDim.x * EW_NT;
  for (int64_t p = (int64_t)blockIdx.x * EW_NT + threadIdx.x; p < Nl; p += stride)
    out[p] = plane_sum(planes, w, G, Nl, p);
}

hipError_t launch_sum_planes(const float* planes, const float* w, int G, int64_t Nl, float* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(sum_planes_kernel, dim3(ew_blocks(Nl)), dim3(EW_NT), 0, s, planes, w, G, Nl,
                     out);
  return hipGetLastError();
}

// Multiplicative update of Eq. (2) from G partial planes of Dn (summed in
// order, weighted as in plane_sum when w != nullptr), with the non-negativity
// clamp and the 0/0 guards; FP64 partials of ||x_new - x||^2 and ||x||^2 (if
// part != nullptr).
__global__ __launch_bounds__(EW_NT) void update_kernel(const float* planes, const float* w, int G,
                                                       int64_t Nl, const float* B, float* x,
                                                       double* part) {
  __shared__ double red[2 * EW_NT / 64];
  const int64_t stride = (int64_t)gridDim.x * EW_NT;
  double dsq = 0.0, xsq = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * EW_NT + threadIdx.x; p < Nl; p += stride) {
    const float Dn = plane_sum(planes, w, G, Nl, p);
    const float xo = x[p];
    const float xn = em_update_value(xo, B[p], Dn);
    x[p] = xn;
    const double d = (double)xn - (double)xo;
    dsq += d * d;
    xsq += (double)xo * (double)xo;
  }
  if (part != nullptr) {
    const double s1 = block_sum<EW_NT>(dsq, red);
    __syncthreads();
    const double s2 = block_sum<EW_NT>(xsq, red + EW_NT / 64);
    if (threadIdx.x == 0) {
      part[2 * blockIdx.x] = s1;
      part[2 * blockIdx.x + 1] = s2;
    }
  }
}

hipError_t launch_update(const float* planes, const float* w, int G, int64_t Nl, const float* B,
                         float* x, double* part, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(blocks), dim3(EW_NT), 0, s, planes, w, G, Nl, B, x, part);
  return hipGetLastError();
}

// FP64 partial sums of u (y - m)^2 over observed pixels (u > 0), one per block:
// the quadratic term of l(x) (Eq. (1)) from a raw model m = F_t x.
__global__ __launch_bounds__(EW_NT) void loglik_partials_kernel(const float* m, const float* u,
                                                                const float* y, int64_t count,
                                                                double* part) {
  __shared__ double red[EW_NT / 64];
  const int64_t stride = (int64_t)gridDim.x * EW_NT;
  double acc = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * EW_NT + threadIdx.x; p < count; p += stride) {
    const float uu = u[p];
    if (uu > 0.f) {
      const double d = (double)y[p] - (double)m[p];
      acc += (double)uu * d * d;
    }
  }
  const double s = block_sum<EW_NT>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t launch_loglik_partials(const float* m, const float* u, const float* y, int64_t count,
                                  double* part, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(loglik_partials_kernel, dim3(blocks), dim3(EW_NT), 0, s, m, u, y, count,
                     part);
  return hipGetLastError();
}

// One block: trace_ll[it] = -1/2 (sum partials + lconst), trace_rc[it] =
// sqrt(sum d^2) / sqrt(sum x^2), it = counters[0]++ (bounded by TRACE_CAP).
__global__ __launch_bounds__(EW_NT) void finalize_iter_kernel(const double* pll, int nll,
                                                              const double* prc, int nrc,
                                                              const double* sc, double* tll,
                                                              double* trc, int* counters) {
  __shared__ double red[EW_NT / 64];
  double ll = 0.0, a = 0.0, b = 0.0;
  if (pll != nullptr) ll = ordered_sum(pll, nll, 1, red);
  __syncthreads();
  if (prc != nullptr) {
    a = ordered_sum(prc, nrc, 2, red);
    __syncthreads();
    b = ordered_sum(prc + 1, nrc, 2, red);
  }
  if (threadIdx.x == 0) {
    const int it = counters[0];
    if (it < TRACE_CAP) {
      if (pll != nullptr) tll[it] = -0.5 * (ll + sc[S_LCONST]);
      if (prc != nullptr) trc[it] = b > 0.0 ? sqrt(a) / sqrt(b) : 0.0;
    }
    counters[0] = it + 1;
  }
}

hipError_t launch_finalize_iter(const double* part_ll, int n_ll, const double* part_rc, int n_rc,
                                const double* scalars, double* trace_ll, double* trace_rc,
                                int* counters, hipStream_t s) {
  hipLaunchKernelGGL(finalize_iter_kernel, dim3(1), dim3(EW_NT), 0, s, part_ll, n_ll, part_rc,
                     n_rc, scalars, trace_ll, trace_rc, counters);
  return hipGetLastError();
}

__global__ __launch_bounds__(EW_NT) void finalize_loglik_kernel(const double* pll, int nll,
                                                                double* sc) {
  __shared__ double red[EW_NT / 64];
  const double ll = ordered_sum(pll, nll, 1, red);
  if (threadIdx.x == 0) sc[S_LOGLIK] = -0.5 * (ll + sc[S_LCONST]);
}

hipError_t launch_finalize_loglik(const double* part_ll, int n_ll, double* scalars,
                                  hipStream_t s) {
  hipLaunchKernelGGL(finalize_loglik_kernel, dim3(1), dim3(EW_NT), 0, s, part_ll, n_ll, scalars);
  return hipGetLastError();
}

__global__ void reset_counters_kernel(int* counters) {
  if (threadIdx.x < 4) counters[threadIdx.x] = 0;
}

hipError_t launch_reset_counters(int* counters, hipStream_t s) {
  hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, s, counters);
  return hipGetLastError();
}

__global__ __launch_bounds__(EW_NT) void copy_kernel(const float* src, float* dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * EW_NT;
  for (int64_t p = (int64_t)blockIdx.x * EW_NT + threadIdx.x; p < count; p += stride)
    dst[p] = src[p];
}

// Flux-sharing replication of frame pixels into factor x factor blocks (the
// up-sampled exposures of the super-resolution run after Eq. (4)); one thread
// per fine pixel, grid-stride.
__global__ __launch_bounds__(256) void upsample_kernel(const float* __restrict__ y,
                                                       const float* __restrict__ v, int64_t count,
                                                       int Hf, int Wf, int f, float* __restrict__ yu,
                                                       float* __restrict__ vu) {
  const int Hu = f * Hf, Wu = f * Wf;
  const float d2 = (float)(f * f), d4 = (float)(f * f * f * f);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const int64_t t = i / ((int64_t)Hu * Wu);
    const int64_t rem = i - t * Hu * Wu;
    const int I = (int)(rem / Wu), J = (int)(rem - (int64_t)I * Wu);
    const int64_t src = (t * Hf + I / f) * Wf + J / f;
    yu[i] = y[src] / d2;
    vu[i] = v[src] / d4;
  }
}

hipError_t launch_upsample(const float* y, const float* v, int n, int Hf, int Wf, int f,
                           float* yu, float* vu, hipStream_t s) {
  const int64_t count = (int64_t)n * f * Hf * f * Wf;
  const int blocks = (int)std::min<int64_t>(8192, (count + 255) / 256);
  hipLaunchKernelGGL(upsample_kernel, dim3(blocks), dim3(256), 0, s, y, v, count, Hf, Wf, f, yu,
                     vu);
  return hipGetLastError();
}

hipError_t launch_copy(const float* src, float* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(ew_blocks(count)), dim3(EW_NT), 0, s, src, dst, count);
  return hipGetLastError();
}

}  // namespace em
