// em_device.h -- small device helpers shared by the HIP sources of libem.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace em {

// LDS column pitch (floats) for tiles stored transposed (one image column per
// LDS row): at least `need`, a multiple of 4 (16-byte reads) with pitch/4 odd,
// so that 16-byte reads of eight consecutive lanes at consecutive columns hit
// distinct bank groups.
__host__ __device__ constexpr int lds_pitch(int need) {
  return (((need + 3) / 4) % 2 == 1) ? ((need + 3) / 4) * 4 : ((need + 3) / 4) * 4 + 4;
}

// Column owned by a lane in the FP32 kernels.  A ds_read_b128 serves lanes
// {0-7, 16-23} (and {8-15, 24-31}, ...) together; mapping each such group to 16
// consecutive columns makes their 16-byte reads of a transposed tile (one
// column per LDS row, odd pitch/4) fall on distinct banks.  A bijection of
// 0..63.
__device__ inline int lane_column(int lane) {
  return (lane & 7) | ((lane >> 4) << 3) | (((lane >> 3) & 1) << 5);
}

// Read-only view of a global buffer through the constant address space: loads
// with wave-uniform addresses are then selected as scalar (s_load) loads, so
// convolution taps arrive in SGPRs.  Only for data no kernel of the same launch
// writes.
typedef __attribute__((address_space(4))) const float* cfloat_ptr;
__device__ inline cfloat_ptr as_const(const float* p) { return (cfloat_ptr)(p); }

// The multiplicative update of Eq. (2) for one latent pixel, with the
// non-negativity clamp and the guards: a zero stays zero (never 0 * inf); a
// pixel no weighted frame pixel sees (Dn = 0) keeps its value; otherwise the
// ratio q = max(B, 0) / Dn is formed first and then applied, x * q.  Every
// kernel that updates x calls this one function, so the rule is the same bit
// for bit in all of them.
__device__ inline float em_update_value(float xo, float Bv, float Dn) {
  if (xo == 0.f) return 0.f;
  if (Dn == 0.f) return xo;
  const float q = fmaxf(Bv, 0.f) / Dn;
  return xo * q;
}

// FP64 sum over a wave of 64 lanes; the result is valid in lane 0.  The
// reduction tree is fixed, so the result is reproducible bit for bit.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// FP64 sum over a block of NT threads; valid in thread 0.  `sh` holds NT/64
// doubles of LDS.  Waves are added in index order.
template <int NT>
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += sh[i];
  }
  return s;
}

}  // namespace em
