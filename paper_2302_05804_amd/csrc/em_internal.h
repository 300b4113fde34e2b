// em_internal.h -- declarations shared inside libem.so (not installed).
//
// Plan of one EM iteration (Eq. (2) of arXiv:2302.05804, Sec. 2) on the GPU:
//   forward  : r_t = u_t (.) F_t x  for every frame t      (+ FP64 l(x) partials)
//   adjoint  : Dn  = sum_t F_t^T r_t                         (fixed frame order)
//   update   : x  <- x (.) max(B,0) / Dn                     (+ FP64 change partials)
// F_t x = D(f_t * x) is a direct K x K convolution (sr = 1) or a stride-2
// convolution with the 2x2-box-extended kernel k_t = h_t * 1_{2x2} of size
// (K+1) x (K+1) (sr = 2, Eq. (3)).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "em.h"

namespace em {

// Supported padded kernel sizes.  A smaller odd K is zero-padded symmetrically
// to the next of these, which leaves every sum unchanged (the extra taps
// multiply finite values by +0).
constexpr int KT_SMALL = 15;
constexpr int KT_LARGE = 43;
constexpr int K_MAX = KT_LARGE;

// Coefficient tables: per frame, KC columns of TAB_LD floats, column b holds
// the kernel taps k[0..KC-1][b] (column-major), KC = KT (sr=1) or KT+1 (sr=2).
constexpr int TAB_LD = 48;

// Device trace capacity (iterations per chunk of em_iterate).
constexpr int TRACE_CAP = 4096;

// Scalar slots (double) in the workspace.
enum Scalar {
  S_SUM_UY = 0,     // sum u*y over unmasked frame pixels
  S_SUM_U = 1,      // sum u
  S_LCONST = 2,     // sum_{u>0} ln(2 pi v)
  S_X0 = 3,         // flat starting value
  S_LOGLIK = 4,     // last em_loglik result
  S_RC_NUM = 5,
  S_RC_DEN = 6,
  S_COUNT = 16
};

struct Geometry {
  int n, Hf, Wf, sr, Hl, Wl, K, KT, KC;
  int64_t Nf, Nl;
  int precision, weight_mode;
  float nu;   // Student-t degrees of freedom (EM_W_STUDENT_T)
};

// Launch shape chosen for a geometry (a pure function of the geometry, so the
// arithmetic of a job never depends on what else runs).
struct Plan {
  // forward
  int fwd_variant;
  int fwd_tiles;       // frame-grid tiles
  int fwd_groups;      // frame groups (grid.y)
  int fwd_fpg;         // frames per group
  // adjoint
  int adj_variant;
  int adj_tiles;       // latent-grid tiles
  int adj_groups;      // frame groups
  int adj_fpg;
  int adj_fused;       // 1 => update fused into the adjoint (one frame group and
                       // the weights on the frame grid); else partial planes
  int lo_band;         // BF16 split: PSF lo part on the central kernel rows only
  // reductions
  int prep_blocks;     // blocks of the per-pixel prep kernel
  int upd_blocks;      // blocks of the separate update kernel
  int max_partials;    // doubles per partial array
};

// Workspace layout (byte offsets from the workspace base, 256-aligned).
struct Layout {
  size_t u, r, ry, B, planes, tab, mtab_fwd, mtab_adj, tune, part_ll, part_rc, part_prep,
      scalars, trace_ll, trace_rc, counters, r16, r16stat, total;
};

// true when the convolutions of geometry g run on the matrix cores
inline bool uses_mfma(const Geometry& g) {
  return g.precision == EM_BF16_SPLIT || g.precision == EM_FP16_SPLIT || g.precision == EM_BF16;
}

bool make_geometry(const void* problem, Geometry* g, const char** why);
Plan make_plan(const Geometry& g);
Layout make_layout(const Geometry& g, const Plan& pl);

// ---- launchers (em_fp32.hip / em_elem.hip) --------------------------------
struct FwdLaunch {
  const float* x;      // latent image
  const float* tab;    // coefficient tables
  const float* u;      // weights (nullptr => raw F_t x output)
  const float* y;      // exposures (loglik only)
  float* out;          // r_t = u_t F_t x  (or F_t x when u == nullptr)
  double* part;        // loglik partials (nullptr => none)
  int n, Hf, Wf, Hl, Wl, fpg;
  int ntiles;          // tiles of the job (partial index = group * ntiles + tile)
  // Student-t noise (out_y != nullptr): out = u w F_t x, out_y = u w y with the
  // E-step weight w = (nu + 1) / (nu + u (y - F_t x)^2); loglik partials of
  // (nu + 1) ln(1 + u (y - F_t x)^2 / nu) - lcst
  float* out_y;
  float nu;
  double lcst;
};

struct AdjLaunch {
  const float* in;     // frame-grid images, n x Nf
  const float* tab;
  float* plane;        // output planes (mode 0), G x Nl
  float* x;            // iterate (fused update)
  const float* B;      // numerator (fused update)
  double* part;        // change partials (fused update, may be nullptr)
  int n, Hf, Wf, Hl, Wl, fpg;
  int fused;           // 1 => x update in the epilogue (G == 1)
  int ntiles;
};

// Matrix-core correlation kernels (em_mfma.hip), sr = 1.
struct MfmaLaunch {
  const float* in;     // forward: x; adjoint: r images (n x H x W)
  const void* tab;     // Toeplitz fragment tables of the direction
  const float* u;      // forward: weights (nullptr => raw output)
  const float* y;      // forward: exposures (loglik)
  float* out;          // forward output
  double* part;        // forward: loglik partials; adjoint: change partials
  float* plane;        // adjoint output planes
  float* x;            // adjoint fused update
  const float* B;
  int n, H, W, fpg;
  int fused;
  int ntiles;
  float* out_y;        // forward under Student-t noise (as FwdLaunch)
  float nu;
  double lcst;
  // binary16 r planes (FP16 split form, sr = 1, Gaussian weights; nullptr =>
  // FP32 r in out / in): the forward writes 2^e16[t] u F x there and the
  // adjoint copies its windows straight into LDS.  Frame t's plane starts at
  // r16 + t * s16 halves; frame pixel (k, l) sits at row k + c, column l + c
  // of rows of p16 halves, c = (KT - 1) / 2; the rest of the plane is zero.
  unsigned short* r16;
  const int* e16;
  int p16;
  int64_t s16;
  // BF16 split, K = 43: the PSF's lo part on the central kernel rows only (the
  // job's PSFs passed the band check at set-up)
  int lo_band;
};
// BF16 split, sr = 1, K = 43: counts in *flag the frames whose PSF keeps more
// than 1/16 of its mass outside the kernel rows that take the lo part
hipError_t launch_lo_band_check(const Geometry& g, const float* psf, int* flag, hipStream_t s);
// sr = 2 split-form forward with the frames in the N dimension of the products
// (em_mfma2n.hip): 16 x m2n_tile_w frame pixels and 16 frames per workgroup,
// jobs of at least M2N_MIN_FRAMES frames
constexpr int M2N_TH = 16, M2N_FPG = 16, M2N_MIN_FRAMES = 8;
// FP16 split 64; BF16 split 32 (its two image planes double the register window)
__host__ __device__ constexpr int m2n_tile_w(int precision) {
  return precision == EM_BF16_SPLIT ? 32 : 64;
}
inline bool uses_m2n(const Geometry& g) {
  return g.sr == 2 && (g.precision == EM_FP16_SPLIT || g.precision == EM_BF16_SPLIT) &&
         g.n >= M2N_MIN_FRAMES;
}
// binary16 r plane geometry.  sr = 1: frame pixel (k, l) at plane (k + c, l + c),
// c = (KT - 1) / 2, so every adjoint window of 128 x 128 outputs (rows k0 - c ..
// k0 + 127 + c, columns l0 - c .. l0 + 175 - c) lies inside the plane and starts
// on a 16-byte boundary.  sr = 2: frame pixel (I, J) at plane (I + 11, J + 11),
// so the window of a 128 x 256 latent tile (96 frame rows of 176 from frame
// (K0/2 - 11, L0/2 - 11)) starts at plane (K0/2, L0/2).
int r16_pitch(const Geometry& g);   // sr = 1: 128 ceil(W / 128) + 48; sr = 2: 128 ceil(Wl / 256) + 48
int r16_rows(const Geometry& g);    // sr = 1: 128 ceil(H / 128) + KT - 1; sr = 2: 64 ceil(Hl / 128) + 32
int r16_off(const Geometry& g);     // c (sr = 1) or 11 (sr = 2)
// Gaussian FP16 split iterations run on binary16 r planes: every sr = 1 job, and
// sr = 2 jobs whose forward has the frames in N
inline bool uses_r16(const Geometry& g) {
  return g.precision == EM_FP16_SPLIT && g.weight_mode == EM_W_ADJOINT &&
         (g.sr == 1 || uses_m2n(g));
}
// set-up of the binary16 r planes: zero planes, per-frame max u and sum of the PSF
hipError_t launch_r16_setup(const Geometry& g, const float* u, const float* psf,
                            unsigned short* r16, float* umax, float* fsum, hipStream_t s);
// per iteration, before the forward: e16[t] from the bound 2 max u_t sum f_t max x
// (max x from `nb` block partials in xpart)
constexpr int R16_XBLOCKS = 256;
hipError_t launch_r16_scale(const Geometry& g, const float* x, float* xpart, const float* umax,
                            const float* fsum, int* e16, hipStream_t s);
// the scale step of several jobs' r16 planes in one pair of launches (serving)
struct R16Job {
  const float* x;
  int64_t Nl;
  float* xpart;
  const float* umax;
  const float* fsum;
  int* e16;
  int n;
};
hipError_t launch_r16_scale_batched(const R16Job* jobs, int n_jobs, hipStream_t s);
hipError_t launch_mfma(const Geometry& g, int dir, int variant, int tiles, int groups,
                       const MfmaLaunch& a, hipStream_t s);
int mfma_table_rows(int KT);
// sr = 2 matrix-core kernels (em_mfma2.hip); K <= 43 padded to 43
hipError_t launch_mfma2(const Geometry& g, int dir, int variant, int tiles, int groups,
                        const MfmaLaunch& a, hipStream_t s);
hipError_t launch_mfma2_batched(int precision, int dir, int variant, const MfmaLaunch* descs,
                                const int4* items, int n_items, int grid, hipStream_t s,
                                bool robust = false, bool m2n = false, bool r16 = false);
hipError_t launch_mfma2_tables(const Geometry& g, const float* psf, void* tab_fwd, void* tab_adj,
                               hipStream_t s);
size_t mfma2_table_bytes(int n, int dir);
size_t mfma2n_table_bytes(int n);
hipError_t launch_mfma2n_table(const Geometry& g, const float* psf, void* tab, hipStream_t s);
hipError_t launch_mfma2n(const Geometry& g, int variant, int tiles, int groups,
                         const MfmaLaunch& a, hipStream_t s);
hipError_t launch_mfma2n_batched(int precision, int variant, const MfmaLaunch* descs,
                                 const int4* items, int n_items, int grid, hipStream_t s,
                                 bool robust);
bool mfma2n_desc_ok(const Geometry& g, int tiles, int groups, const MfmaLaunch& a);
int mfma2_fwd_tile_h(int precision);
int mfma2_fwd_tile_w(int precision);
int mfma2_adj_tile_h(int precision);
int mfma2_adj_tile_w(int precision);
hipError_t launch_mfma_batched(int KT, int precision, int dir, int variant, const MfmaLaunch* descs,
                               const int4* items, int n_items, int grid, hipStream_t s,
                               bool robust = false, bool r16 = false);
// 2 (lgamma((nu+1)/2) - lgamma(nu/2) - ln(nu pi)/2) + ln(2 pi): the constant of
// the Student-t loglik partials (em_api.cpp)
double student_t_lcst(double nu);
hipError_t launch_forward_batched(int sr, int KT, const FwdLaunch* descs, const int4* items,
                                  int n_items, int grid, hipStream_t s);
hipError_t launch_adjoint_batched(int sr, int KT, const AdjLaunch* descs, const int4* items,
                                  int n_items, int grid, hipStream_t s);
int mfma_variants();
hipError_t launch_mfma_tables(const Geometry& g, const float* psf, void* tab_fwd, void* tab_adj,
                              hipStream_t s);
int mfma_tile_h();
int mfma_tile_w();
size_t mfma_table_bytes(const Geometry& g, int dir);

// Host-side check that a launch grid matches its descriptor: `tiles` tiles of
// tile_h x tile_w cover an h x w grid exactly, and `groups` frame groups of fpg
// frames cover n frames exactly.  Launchers refuse anything else, so a
// descriptor built for the wrong grid is an error, never an out-of-range access.
inline bool launch_grid_ok(int tiles, int groups, int ntiles, int n, int fpg, int h, int w,
                           int tile_h, int tile_w) {
  if (h < 1 || w < 1 || n < 1 || fpg < 1 || groups < 1 || tiles < 1) return false;
  const int64_t expect = (int64_t)((w + tile_w - 1) / tile_w) * ((h + tile_h - 1) / tile_h);
  return tiles == expect && ntiles == tiles && (int64_t)groups * fpg >= n &&
         (int64_t)(groups - 1) * fpg < n;
}

bool forward_desc_ok(const Geometry& g, int tiles, int groups, const FwdLaunch& a);
bool adjoint_desc_ok(const Geometry& g, int tiles, int groups, const AdjLaunch& a);
bool mfma_desc_ok(const Geometry& g, int dir, int tiles, int groups, const MfmaLaunch& a);
bool mfma2_desc_ok(const Geometry& g, int dir, int tiles, int groups, const MfmaLaunch& a);

hipError_t launch_forward(const Geometry& g, const Plan& pl, const FwdLaunch& a, hipStream_t s);
hipError_t launch_adjoint(const Geometry& g, const Plan& pl, const AdjLaunch& a, hipStream_t s);

struct PrepLaunch {
  const float* y;
  const float* v;
  float* u;
  float* w;            // u * y, or y alone when raw_y (masked y -> 0 in both)
  int raw_y;
  double* part;        // 3 x blocks partial sums
  int* flags;          // [0] invalid data count
  int64_t count;       // n * Nf
  int blocks;
};
hipError_t launch_prep(const PrepLaunch& a, hipStream_t s);

hipError_t launch_psf_tables(const Geometry& g, const float* psf, float* tab, int* flags,
                             hipStream_t s);

// FP64 partials of sum_{u>0} u (y - m)^2 over `count` frame pixels, one per
// block (`blocks` of them), for forwards that write the raw model m = F_t x.
hipError_t launch_loglik_partials(const float* m, const float* u, const float* y, int64_t count,
                                  double* part, int blocks, hipStream_t s);
// sums `count` partials of `nsum` interleaved arrays in fixed order
hipError_t launch_finalize_prep(const double* part, int blocks, double* scalars, int sr,
                                hipStream_t s);
hipError_t launch_init_x(const float* x0, float* x, const double* scalars, int64_t count,
                         int* flags, hipStream_t s);
// out = sum_g planes[g] (times w[g] when w != nullptr: the per-frame weights of
// the typeset form of Eq. (2), G = n), in order g = 0..G-1
hipError_t launch_sum_planes(const float* planes, const float* w, int G, int64_t Nl, float* out,
                             hipStream_t s);
hipError_t launch_update(const float* planes, const float* w, int G, int64_t Nl, const float* B,
                         float* x, double* part, int blocks, hipStream_t s);
// iteration bookkeeping: writes trace entries at counters[0] and advances it
hipError_t launch_finalize_iter(const double* part_ll, int n_ll, const double* part_rc,
                                int n_rc, const double* scalars, double* trace_ll,
                                double* trace_rc, int* counters, hipStream_t s);
hipError_t launch_finalize_loglik(const double* part_ll, int n_ll, double* scalars,
                                  hipStream_t s);
hipError_t launch_reset_counters(int* counters, hipStream_t s);
hipError_t launch_copy(const float* src, float* dst, int64_t count, hipStream_t s);
hipError_t launch_upsample(const float* y, const float* v, int n, int Hf, int Wf, int f,
                           float* yu, float* vu, hipStream_t s);

// Super-resolved PSFs of Eq. (4) (em_psf.hip): one workgroup per frame.
constexpr int PSF_K_MAX = 63;
struct PsfParams {
  int n, kf, kh, D, S;
  float sigma, lam, lr, decay, b1, b2, eps;
};
size_t psf_lds_bytes(int kf, int kh);
hipError_t launch_psf_fit(const PsfParams& P, const float* f, const float* h0, float* h,
                          double* objective, hipStream_t s);

}  // namespace em

// One deconvolution job (opaque in the C ABI).
struct em_ctx {
  em::Geometry g;
  em::Plan pl;
  em::Layout lay;
  hipStream_t stream;
  const float* y;
  const float* v;
  const float* psf;
  float* x;
  char* ws;
  // device views into the workspace
  float* u;
  float* r;
  float* ry;   // u w y of the Student-t iteration (EM_W_STUDENT_T only)
  float* B;
  float* planes;
  float* tab;
  void* mtab_fwd;
  void* mtab_adj;
  float* tune;
  double* part_ll;
  double* part_rc;
  double* part_prep;
  double* scalars;
  double* trace_ll;
  double* trace_rc;
  int* counters;  // [0] iteration counter, [4..7] validation flags
  // binary16 r planes (uses_r16): planes, then umax[n], fsum[n] (float),
  // e16[n] (int), xpart[R16_XBLOCKS] (float)
  unsigned short* r16;
  float* r16_umax;
  float* r16_fsum;
  int* r16_e;
  float* r16_xpart;
  // captured iteration (em_iterate without / with the FP64 trace bookkeeping)
  hipGraphExec_t graph[2];
  bool graph_ok[2];
  bool no_graph;  // iterations always launched eagerly (nothing instantiated)
};


void em_bind_views(em_ctx* c);
namespace em {
int fail(int code, const char* fmt, ...);
// fill the launch descriptors of ctx's forward / adjoint (fused update) passes
void fill_forward_fp32(const em_ctx* c, FwdLaunch* f, bool write_r, bool loglik);
void fill_forward_mfma(const em_ctx* c, MfmaLaunch* m, bool write_r, bool loglik);
void fill_adjoint_fp32(const em_ctx* c, AdjLaunch* a, double* part_rc);
void fill_adjoint_mfma(const em_ctx* c, MfmaLaunch* m, double* part_rc);
// point a forward (dir 0) or adjoint (dir 1) descriptor at the job's binary16 r planes
void apply_r16(const em_ctx* c, MfmaLaunch* m, int dir);
// em_init with the plan used by the serving loop (single frame group in the
// adjoint, fixed kernel variants), so a served job computes the same way
// alone and in any mix.
int init_ctx(em_ctx** out, const em_problem* p, const float* y, const float* v, const float* psf,
             const float* x0, float* x, void* workspace, size_t ws_bytes, void* stream,
             bool serving);
Plan make_serving_plan(const Geometry& g);
}  // namespace em
