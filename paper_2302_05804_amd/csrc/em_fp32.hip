// em_fp32.hip -- FP32 direct-convolution kernels of one EM iteration
// (arXiv:2302.05804, Sec. 2: forward model of Eq. (1) / Eq. (3), weighting and
// adjoint of Eq. (2)).
//
// All four kernels share one scheme, chosen for CDNA4's 64-wide waves:
//  * a workgroup stages an input tile plus its K-1 halo in LDS, stored
//    transposed (one image column per LDS row), so that a lane reads a whole
//    column segment with 16-byte ds_read_b128;
//  * lane l owns one output column and a strip of R consecutive output rows;
//    per kernel column b it loads the column segment into registers and applies
//    the K taps of column b, which are wave-uniform and therefore come from
//    scalar registers (s_load from the coefficient table);
//  * R*K FMAs per R+K-1 LDS values keeps the kernels VALU-bound;
//  * sums are formed in levels (one kernel column, then one frame, then the
//    total), which keeps the FP32 rounding error of a K*K*n-term sum near that
//    of its ~K-term pieces instead of growing with the full chain.
// The forward kernels loop over frames inside the workgroup (x is shared by all
// frames, its tile is loaded once); the adjoint kernels loop over frames with
// the per-pixel sum over frames held in registers (fixed frame order, no
// atomics), and either write a partial plane per frame group or apply the
// multiplicative update in the epilogue.
#include "em_device.h"
#include "em_internal.h"

namespace em {

// Forward epilogue of one output: m = F_t x raw (u == nullptr); r = u m and
// the FP64 partial of u (y - m)^2; or, under Student-t noise (out_y), r = u w m,
// out_y = u w y with w = (nu + 1) / (nu + u (y - m)^2), and the partial of
// (nu + 1) ln(1 + u (y - m)^2 / nu) - lcst.
__device__ inline void fwd_store(const FwdLaunch& a, int64_t idx, float m, double& llp) {
  if (a.u == nullptr) {
    a.out[idx] = m;
    return;
  }
  const float uu = a.u[idx];
  if (a.out_y != nullptr) {
    float ro = 0.f, ryo = 0.f;
    if (uu > 0.f) {
      const float y = a.y[idx];
      const float d = y - m;
      const float w = (a.nu + 1.f) / (a.nu + uu * d * d);
      ro = (uu * w) * m;
      ryo = (uu * w) * y;
      if (a.part != nullptr) {
        const double dd = (double)y - (double)m;
        llp += ((double)a.nu + 1.0) * log1p((double)uu * dd * dd / (double)a.nu) - a.lcst;
      }
    }
    a.out[idx] = ro;
    a.out_y[idx] = ryo;
    return;
  }
  if (a.out) a.out[idx] = uu * m;
  if (a.part != nullptr && uu > 0.f) {
    const double d = (double)a.y[idx] - (double)m;
    llp += (double)uu * d * d;
  }
}

// ---------------------------------------------------------------------------
// sr = 1 forward:  m_t[i,j] = sum_{a,b} f_t[a,b] x[i+c-a, j+c-b]      (Eq. (1))
//   epilogue: r_t = u_t m_t (or m_t raw), FP64 partial of u (y - m)^2.
// ---------------------------------------------------------------------------
template <int KT, int R, int WV>
__device__ inline void fwd1_body(const FwdLaunch& a, const int tile, const int group) {
  constexpr int c = (KT - 1) / 2;
  constexpr int TW = 64, TH = R * WV;
  constexpr int LW = TW + KT - 1;
  constexpr int NR = R + KT - 1;
  constexpr int NR4 = (NR + 3) / 4 * 4;
  constexpr int P = lds_pitch((WV - 1) * R + NR4);
  constexpr int LH = TH + KT - 1;
  __shared__ __align__(16) float xs[LW * P];
  __shared__ double red[WV];

  const int lane = lane_column(threadIdx.x & 63), w = threadIdx.x >> 6;
  const int tiles_x = (a.Wf + TW - 1) / TW;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int j0 = tx * TW, i0 = ty * TH;

  for (int e = threadIdx.x; e < LW * P; e += 64 * WV) {
    const int row = e / LW, col = e - row * LW;
    const int gy = i0 - c + row, gx = j0 - c + col;
    float val = 0.f;
    if (row < LH && gy >= 0 && gy < a.Hl && gx >= 0 && gx < a.Wl)
      val = a.x[(int64_t)gy * a.Wl + gx];
    xs[col * P + row] = val;
  }
  __syncthreads();

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const int64_t Nf = (int64_t)a.Hf * a.Wf;
  const int j = j0 + lane;
  double llp = 0.0;
  for (int t = t0; t < t1; ++t) {
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.f;
    cfloat_ptr tb = as_const(a.tab) + (int64_t)t * KT * TAB_LD;
    for (int b = 0; b < KT; ++b) {
      const float* col = xs + (lane + KT - 1 - b) * P + w * R;
      float xc[NR4];
#pragma unroll
      for (int q = 0; q < NR4; q += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(col + q);
        xc[q] = v4.x; xc[q + 1] = v4.y; xc[q + 2] = v4.z; xc[q + 3] = v4.w;
      }
      cfloat_ptr fb = tb + b * TAB_LD;
      float part[R];   // two-level sum: one kernel column, then the total
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = 0.f;
#pragma unroll
      for (int aa = 0; aa < KT; ++aa) {
        const float fv = fb[aa];
#pragma unroll
        for (int r = 0; r < R; ++r) part[r] = fmaf(fv, xc[r + KT - 1 - aa], part[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += part[r];
    }
    if (j < a.Wf) {
      const int64_t base = (int64_t)t * Nf;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = i0 + w * R + r;
        if (i < a.Hf) {
          fwd_store(a, base + (int64_t)i * a.Wf + j, acc[r], llp);
        }
      }
    }
  }
  if (a.part != nullptr) {
    const double s = block_sum<64 * WV>(llp, red);
    if (threadIdx.x == 0) a.part[(int64_t)group * a.ntiles + tile] = s;
  }
}

// ---------------------------------------------------------------------------
// sr = 2 forward (Eq. (3)):  m_t[I,J] = sum_{a',b'=0..K} k_t[a',b'] x[2I+c+1-a', 2J+c+1-b']
// with k_t = h_t extended by the 2x2 box.  The x tile is stored as two column
// phases (even / odd latent columns) so that lanes read consecutive LDS rows.
// ---------------------------------------------------------------------------
template <int KT, int R, int WV>
__device__ inline void fwd2_body(const FwdLaunch& a, const int tile, const int group) {
  constexpr int c = (KT - 1) / 2;
  constexpr int KC = KT + 1;
  constexpr int TW = 64, TH = R * WV;          // frame pixels
  constexpr int LWL = 2 * TW + KT - 1;         // latent columns staged
  constexpr int LWP = (LWL + 1) / 2;           // per phase
  constexpr int NR = 2 * R + KT - 1;           // latent rows read per thread
  constexpr int NR4 = (NR + 3) / 4 * 4;
  constexpr int P = lds_pitch(2 * (WV - 1) * R + NR4);
  constexpr int LH = 2 * TH + KT - 1;
  __shared__ __align__(16) float xs[2 * LWP * P];
  __shared__ double red[WV];

  const int lane = lane_column(threadIdx.x & 63), w = threadIdx.x >> 6;
  const int tiles_x = (a.Wf + TW - 1) / TW;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int J0 = tx * TW, I0 = ty * TH;
  const int Y0 = 2 * I0 + c + 1 - KT, X0 = 2 * J0 + c + 1 - KT;

  for (int e = threadIdx.x; e < 2 * LWP * P; e += 64 * WV) {
    const int row = e / (2 * LWP), C = e - row * (2 * LWP);
    const int gy = Y0 + row, gx = X0 + C;
    float val = 0.f;
    if (row < LH && C < LWL && gy >= 0 && gy < a.Hl && gx >= 0 && gx < a.Wl)
      val = a.x[(int64_t)gy * a.Wl + gx];
    xs[((C & 1) * LWP + (C >> 1)) * P + row] = val;
  }
  __syncthreads();

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  const int64_t Nf = (int64_t)a.Hf * a.Wf;
  const int J = J0 + lane;
  double llp = 0.0;
  for (int t = t0; t < t1; ++t) {
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.f;
    cfloat_ptr tb = as_const(a.tab) + (int64_t)t * KC * TAB_LD;
    for (int b = 0; b < KC; ++b) {
      const int ph = (KT - b) & 1;
      const float* col = xs + (ph * LWP + lane + ((KT - b) >> 1)) * P + 2 * w * R;
      float xc[NR4];
#pragma unroll
      for (int q = 0; q < NR4; q += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(col + q);
        xc[q] = v4.x; xc[q + 1] = v4.y; xc[q + 2] = v4.z; xc[q + 3] = v4.w;
      }
      cfloat_ptr fb = tb + b * TAB_LD;
      float part[R];
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = 0.f;
#pragma unroll
      for (int aa = 0; aa < KC; ++aa) {
        const float fv = fb[aa];
#pragma unroll
        for (int r = 0; r < R; ++r) part[r] = fmaf(fv, xc[2 * r + KT - aa], part[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += part[r];
    }
    if (J < a.Wf) {
      const int64_t base = (int64_t)t * Nf;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int I = I0 + w * R + r;
        if (I < a.Hf) {
          fwd_store(a, base + (int64_t)I * a.Wf + J, acc[r], llp);
        }
      }
    }
  }
  if (a.part != nullptr) {
    const double s = block_sum<64 * WV>(llp, red);
    if (threadIdx.x == 0) a.part[(int64_t)group * a.ntiles + tile] = s;
  }
}

// ---------------------------------------------------------------------------
// sr = 1 adjoint: s[k,l] = sum_{a,b} f_t[a,b] r_t[k-c+a, l-c+b], summed over t.
// ---------------------------------------------------------------------------
template <int KT, int R, int WV>
__device__ inline void adj1_body(const AdjLaunch& a, const int tile, const int group) {
  constexpr int c = (KT - 1) / 2;
  constexpr int TW = 64, TH = R * WV;
  constexpr int LW = TW + KT - 1;
  constexpr int NR = R + KT - 1;
  constexpr int NR4 = (NR + 3) / 4 * 4;
  constexpr int P = lds_pitch((WV - 1) * R + NR4);
  constexpr int LH = TH + KT - 1;
  __shared__ __align__(16) float rs[LW * P];
  __shared__ double red[2 * WV];

  const int lane = lane_column(threadIdx.x & 63), w = threadIdx.x >> 6;
  const int tiles_x = (a.Wl + TW - 1) / TW;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int l0 = tx * TW, k0 = ty * TH;
  const int64_t Nf = (int64_t)a.Hf * a.Wf;

  float acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.f;

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  for (int t = t0; t < t1; ++t) {
    const float* src = a.in + (int64_t)t * Nf;
    __syncthreads();
    for (int e = threadIdx.x; e < LW * P; e += 64 * WV) {
      const int row = e / LW, col = e - row * LW;
      const int gy = k0 - c + row, gx = l0 - c + col;
      float val = 0.f;
      if (row < LH && gy >= 0 && gy < a.Hf && gx >= 0 && gx < a.Wf)
        val = src[(int64_t)gy * a.Wf + gx];
      rs[col * P + row] = val;
    }
    __syncthreads();
    cfloat_ptr tb = as_const(a.tab) + (int64_t)t * KT * TAB_LD;
    float facc[R];   // this frame's sum (three-level sum: column, frame, total)
#pragma unroll
    for (int r = 0; r < R; ++r) facc[r] = 0.f;
    for (int b = 0; b < KT; ++b) {
      const float* col = rs + (lane + b) * P + w * R;
      float rc[NR4];
#pragma unroll
      for (int q = 0; q < NR4; q += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(col + q);
        rc[q] = v4.x; rc[q + 1] = v4.y; rc[q + 2] = v4.z; rc[q + 3] = v4.w;
      }
      cfloat_ptr fb = tb + b * TAB_LD;
      float part[R];
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = 0.f;
#pragma unroll
      for (int aa = 0; aa < KT; ++aa) {
        const float fv = fb[aa];
#pragma unroll
        for (int r = 0; r < R; ++r) part[r] = fmaf(fv, rc[r + aa], part[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) facc[r] += part[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += facc[r];
  }

  const int l = l0 + lane;
  double dsq = 0.0, xsq = 0.0;
  if (l < a.Wl) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = k0 + w * R + r;
      if (k < a.Hl) {
        const int64_t idx = (int64_t)k * a.Wl + l;
        if (a.fused) {
          const float xo = a.x[idx];
          const float xn = em_update_value(xo, a.B[idx], acc[r]);
          a.x[idx] = xn;
          const double d = (double)xn - (double)xo;
          dsq += d * d;
          xsq += (double)xo * (double)xo;
        } else {
          a.plane[(int64_t)group * a.Hl * a.Wl + idx] = acc[r];
        }
      }
    }
  }
  if (a.fused && a.part != nullptr) {
    const double s1 = block_sum<64 * WV>(dsq, red);
    __syncthreads();
    const double s2 = block_sum<64 * WV>(xsq, red + WV);
    if (threadIdx.x == 0) {
      a.part[2 * tile] = s1;
      a.part[2 * tile + 1] = s2;
    }
  }
}

// ---------------------------------------------------------------------------
// sr = 2 adjoint (transpose of Eq. (3)'s operator):
//   s[k,l] = sum_{I,J} r_t[I,J] k_t[2I+c+1-k, 2J+c+1-l],  summed over t.
// A wave owns latent columns of one parity (l = l0 + 2*lane + ph), which makes
// every tap wave-uniform.  With h = (c+1)/2 (c odd for the supported sizes):
//   J = l0/2 + lane + dd + ph - h   -> b' = 2 dd + ph,   dd in [0, 2h)
//   I = k0/2 + w R/2 + e - h        -> a' = 2 e - rr,    rr = row in strip
// ---------------------------------------------------------------------------
template <int KT, int R, int WV>
__device__ inline void adj2_body(const AdjLaunch& a, const int tile, const int group) {
  constexpr int c = (KT - 1) / 2;
  static_assert(c % 2 == 1, "sr=2 adjoint assumes odd c");
  static_assert(R % 8 == 0, "strip height must keep 16-byte LDS alignment");
  constexpr int h = (c + 1) / 2;
  constexpr int KC = KT + 1;
  constexpr int TWL = 128, THL = R * WV;         // latent tile
  constexpr int LW = TWL / 2 + 2 * h;            // frame columns staged
  constexpr int NE = R / 2 + 2 * h;              // frame rows read per thread
  constexpr int NE4 = (NE + 3) / 4 * 4;
  constexpr int P = lds_pitch((WV - 1) * R / 2 + NE4);
  constexpr int LH = THL / 2 + 2 * h;
  constexpr int NT = 128 * WV;
  __shared__ __align__(16) float rs[LW * P];
  __shared__ double red[2 * NT / 64];

  const int lane = lane_column(threadIdx.x & 63), wid = threadIdx.x >> 6;
  const int ph = wid & 1, w = wid >> 1;
  const int tiles_x = (a.Wl + TWL - 1) / TWL;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int l0 = tx * TWL, k0 = ty * THL;
  const int Jb = l0 / 2 - h, Ib = k0 / 2 - h;
  const int64_t Nf = (int64_t)a.Hf * a.Wf;

  float acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.f;

  const int t0 = group * a.fpg;
  const int t1 = min(a.n, t0 + a.fpg);
  for (int t = t0; t < t1; ++t) {
    const float* src = a.in + (int64_t)t * Nf;
    __syncthreads();
    for (int e = threadIdx.x; e < LW * P; e += NT) {
      const int row = e / LW, col = e - row * LW;
      const int gy = Ib + row, gx = Jb + col;
      float val = 0.f;
      if (row < LH && gy >= 0 && gy < a.Hf && gx >= 0 && gx < a.Wf)
        val = src[(int64_t)gy * a.Wf + gx];
      rs[col * P + row] = val;
    }
    __syncthreads();
    cfloat_ptr tb = as_const(a.tab) + (int64_t)t * KC * TAB_LD;
    float facc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) facc[r] = 0.f;
    for (int dd = 0; dd < 2 * h; ++dd) {
      const float* col = rs + (lane + dd + ph) * P + w * (R / 2);
      float rc[NE4];
#pragma unroll
      for (int q = 0; q < NE4; q += 4) {
        const float4 v4 = *reinterpret_cast<const float4*>(col + q);
        rc[q] = v4.x; rc[q + 1] = v4.y; rc[q + 2] = v4.z; rc[q + 3] = v4.w;
      }
      cfloat_ptr fb = tb + (2 * dd + ph) * TAB_LD;
      float fk[KC];
#pragma unroll
      for (int aa = 0; aa < KC; ++aa) fk[aa] = fb[aa];
      float part[R];
#pragma unroll
      for (int r = 0; r < R; ++r) part[r] = 0.f;
#pragma unroll
      for (int e = 0; e < NE; ++e) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int ap = 2 * e - r;
          if (ap >= 0 && ap < KC) part[r] = fmaf(fk[ap], rc[e], part[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) facc[r] += part[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] += facc[r];
  }

  const int l = l0 + 2 * lane + ph;
  double dsq = 0.0, xsq = 0.0;
  if (l < a.Wl) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = k0 + w * R + r;
      if (k < a.Hl) {
        const int64_t idx = (int64_t)k * a.Wl + l;
        if (a.fused) {
          const float xo = a.x[idx];
          const float xn = em_update_value(xo, a.B[idx], acc[r]);
          a.x[idx] = xn;
          const double d = (double)xn - (double)xo;
          dsq += d * d;
          xsq += (double)xo * (double)xo;
        } else {
          a.plane[(int64_t)group * a.Hl * a.Wl + idx] = acc[r];
        }
      }
    }
  }
  if (a.fused && a.part != nullptr) {
    const double s1 = block_sum<NT>(dsq, red);
    __syncthreads();
    const double s2 = block_sum<NT>(xsq, red + NT / 64);
    if (threadIdx.x == 0) {
      a.part[2 * tile] = s1;
      a.part[2 * tile + 1] = s2;
    }
  }
}

// ---------------------------------------------------------------------------
// Entry points.  `*_kernel`: one job, grid (tiles, frame groups).  `*_batched`:
// several jobs in one launch -- each work item names a job descriptor, a tile
// and a frame group; the workgroups stride over the items (persistent loop with
// a fixed bound, so every wave exits).  A job's arithmetic is identical in both.
// ---------------------------------------------------------------------------
#define EM_FP32_ENTRY(NAME, LAUNCH, BOUND)                                                      \
  template <int KT, int R, int WV>                                                             \
  __global__ __launch_bounds__(BOUND) void NAME##_kernel(LAUNCH a) {                           \
    NAME##_body<KT, R, WV>(a, blockIdx.x, blockIdx.y);                                         \
  }                                                                                            \
  template <int KT, int R, int WV>                                                             \
  __global__ __launch_bounds__(BOUND) void NAME##_batched(const LAUNCH* __restrict__ descs,    \
                                                          const int4* __restrict__ items,      \
                                                          int n_items) {                       \
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {                                    \
      const int4 w = items[i];                                                                 \
      const LAUNCH d = descs[w.x];                                                             \
      NAME##_body<KT, R, WV>(d, w.y, w.z);                                                     \
      __syncthreads();                                                                         \
    }                                                                                          \
  }

EM_FP32_ENTRY(fwd1, FwdLaunch, 64 * WV)
EM_FP32_ENTRY(fwd2, FwdLaunch, 64 * WV)
EM_FP32_ENTRY(adj1, AdjLaunch, 64 * WV)
EM_FP32_ENTRY(adj2, AdjLaunch, 128 * WV)

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
// forward variants: {R, WV}
constexpr int F1_R = 16, F1_WV = 4;
constexpr int F2_R = 8, F2_WV = 4;
constexpr int A1_R = 16, A1_WV = 4;
constexpr int A2_R = 16, A2_WV = 4;
}  // namespace

int fwd_tile_h(const Geometry& g) { return g.sr == 1 ? F1_R * F1_WV : F2_R * F2_WV; }
int fwd_tile_w(const Geometry&) { return 64; }
int adj_tile_h(const Geometry& g) { return g.sr == 1 ? A1_R * A1_WV : A2_R * A2_WV; }
int adj_tile_w(const Geometry& g) { return g.sr == 1 ? 64 : 128; }

bool forward_desc_ok(const Geometry& g, int tiles, int groups, const FwdLaunch& a) {
  return a.Hl == g.sr * a.Hf && a.Wl == g.sr * a.Wf &&
         launch_grid_ok(tiles, groups, a.ntiles, a.n, a.fpg, a.Hf, a.Wf, fwd_tile_h(g),
                        fwd_tile_w(g));
}

bool adjoint_desc_ok(const Geometry& g, int tiles, int groups, const AdjLaunch& a) {
  return a.Hl == g.sr * a.Hf && a.Wl == g.sr * a.Wf &&
         launch_grid_ok(tiles, groups, a.ntiles, a.n, a.fpg, a.Hl, a.Wl, adj_tile_h(g),
                        adj_tile_w(g));
}

hipError_t launch_forward(const Geometry& g, const Plan& pl, const FwdLaunch& a, hipStream_t s) {
  if (!forward_desc_ok(g, pl.fwd_tiles, pl.fwd_groups, a)) return hipErrorInvalidValue;
  dim3 grid(pl.fwd_tiles, pl.fwd_groups);
  if (g.sr == 1) {
    dim3 block(64 * F1_WV);
    if (g.KT == KT_LARGE)
      hipLaunchKernelGGL((fwd1_kernel<KT_LARGE, F1_R, F1_WV>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((fwd1_kernel<KT_SMALL, F1_R, F1_WV>), grid, block, 0, s, a);
  } else {
    dim3 block(64 * F2_WV);
    if (g.KT == KT_LARGE)
      hipLaunchKernelGGL((fwd2_kernel<KT_LARGE, F2_R, F2_WV>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((fwd2_kernel<KT_SMALL, F2_R, F2_WV>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const Geometry& g, const Plan& pl, const AdjLaunch& a, hipStream_t s) {
  if (!adjoint_desc_ok(g, pl.adj_tiles, pl.adj_groups, a)) return hipErrorInvalidValue;
  dim3 grid(pl.adj_tiles, pl.adj_groups);
  if (g.sr == 1) {
    dim3 block(64 * A1_WV);
    if (g.KT == KT_LARGE)
      hipLaunchKernelGGL((adj1_kernel<KT_LARGE, A1_R, A1_WV>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((adj1_kernel<KT_SMALL, A1_R, A1_WV>), grid, block, 0, s, a);
  } else {
    dim3 block(128 * A2_WV);
    if (g.KT == KT_LARGE)
      hipLaunchKernelGGL((adj2_kernel<KT_LARGE, A2_R, A2_WV>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((adj2_kernel<KT_SMALL, A2_R, A2_WV>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_forward_batched(int sr, int KT, const FwdLaunch* descs, const int4* items,
                                  int n_items, int grid, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (sr == 1) {
    dim3 block(64 * F1_WV);
    if (KT == KT_LARGE)
      hipLaunchKernelGGL((fwd1_batched<KT_LARGE, F1_R, F1_WV>), dim3(grid), block, 0, s, descs, items, n_items);
    else
      hipLaunchKernelGGL((fwd1_batched<KT_SMALL, F1_R, F1_WV>), dim3(grid), block, 0, s, descs, items, n_items);
  } else {
    dim3 block(64 * F2_WV);
    if (KT == KT_LARGE)
      hipLaunchKernelGGL((fwd2_batched<KT_LARGE, F2_R, F2_WV>), dim3(grid), block, 0, s, descs, items, n_items);
    else
      hipLaunchKernelGGL((fwd2_batched<KT_SMALL, F2_R, F2_WV>), dim3(grid), block, 0, s, descs, items, n_items);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint_batched(int sr, int KT, const AdjLaunch* descs, const int4* items,
                                  int n_items, int grid, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (sr == 1) {
    dim3 block(64 * A1_WV);
    if (KT == KT_LARGE)
      hipLaunchKernelGGL((adj1_batched<KT_LARGE, A1_R, A1_WV>), dim3(grid), block, 0, s, descs, items, n_items);
    else
      hipLaunchKernelGGL((adj1_batched<KT_SMALL, A1_R, A1_WV>), dim3(grid), block, 0, s, descs, items, n_items);
  } else {
    dim3 block(128 * A2_WV);
    if (KT == KT_LARGE)
      hipLaunchKernelGGL((adj2_batched<KT_LARGE, A2_R, A2_WV>), dim3(grid), block, 0, s, descs, items, n_items);
    else
      hipLaunchKernelGGL((adj2_batched<KT_SMALL, A2_R, A2_WV>), dim3(grid), block, 0, s, descs, items, n_items);
  }
  return hipGetLastError();
}

}  // namespace em
