// em_api.cpp -- C ABI of libem.so (declared in include/em.h): problem
// validation, workspace layout, launch planning and the iteration driver of
// the multiplicative EM update (arXiv:2302.05804, Sec. 2, Eq. (2)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/em.h"
#include "em_internal.h"

namespace em {

int fwd_tile_h(const Geometry& g);
int fwd_tile_w(const Geometry& g);
int adj_tile_h(const Geometry& g);
int adj_tile_w(const Geometry& g);

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define EM_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return em::fail(EM_EDEVICE, "%s: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                      __FILE__, __LINE__);                                            \
  } while (0)

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool make_geometry(const void* problem, Geometry* g, const char** why) {
  const em_problem* p = static_cast<const em_problem*>(problem);
  if (!p) { *why = "problem is NULL"; return false; }
  if (p->n_frames < 1) { *why = "n_frames must be >= 1"; return false; }
  if (p->frame_h < 1 || p->frame_w < 1) { *why = "frame size must be >= 1"; return false; }
  if (p->frame_h > 65536 || p->frame_w > 65536) { *why = "frame side above 65536"; return false; }
  if (p->psf_k < 1 || p->psf_k % 2 == 0 || p->psf_k > K_MAX) {
    *why = "psf_k must be odd and in [1, 43]";
    return false;
  }
  if (p->sr != 1 && p->sr != 2) { *why = "sr must be 1 or 2"; return false; }
  if (p->weight_mode != EM_W_ADJOINT && p->weight_mode != EM_W_LITERAL &&
      p->weight_mode != EM_W_STUDENT_T) {
    *why = "unknown weight_mode";
    return false;
  }
  if (p->weight_mode == EM_W_STUDENT_T && !(p->nu > 0.f && p->nu <= 1e30f)) {
    *why = "nu must be in (0, 1e30] for Student-t noise";
    return false;
  }
  if (p->precision < EM_FP32 || p->precision > EM_BF16) { *why = "unknown precision"; return false; }
  g->n = p->n_frames;
  g->Hf = p->frame_h;
  g->Wf = p->frame_w;
  g->sr = p->sr;
  g->Hl = p->frame_h * p->sr;
  g->Wl = p->frame_w * p->sr;
  g->K = p->psf_k;
  g->KT = p->psf_k <= KT_SMALL ? KT_SMALL : KT_LARGE;
  g->KC = g->sr == 1 ? g->KT : g->KT + 1;
  g->Nf = (int64_t)g->Hf * g->Wf;
  g->Nl = (int64_t)g->Hl * g->Wl;
  g->precision = p->precision;
  g->weight_mode = p->weight_mode;
  g->nu = p->weight_mode == EM_W_STUDENT_T ? p->nu : 0.f;
  if ((int64_t)g->n * g->Nf > ((int64_t)1 << 40)) { *why = "problem too large"; return false; }
  if (g->Nl >= ((int64_t)1 << 31)) { *why = "latent image of 2^31 pixels or more"; return false; }
  return true;
}

Plan make_plan(const Geometry& g) {
  Plan pl{};
  // ~4 workgroups per compute unit on 256 CUs (matrix-core kernels: one
  // workgroup fills a compute unit's LDS, aim for 2 rounds)
  const int target = uses_mfma(g) ? 512 : 1024;
  pl.fwd_variant = 0;
  const bool mf = uses_mfma(g);
  if (uses_m2n(g))
    pl.fwd_tiles = (int)(cdiv(g.Wf, m2n_tile_w(g.precision)) * cdiv(g.Hf, M2N_TH));
  else if (mf && g.sr == 2)
    pl.fwd_tiles = (int)(cdiv(g.Wf, mfma2_fwd_tile_w(g.precision)) *
                         cdiv(g.Hf, mfma2_fwd_tile_h(g.precision)));
  else if (mf)
    pl.fwd_tiles = (int)(cdiv(g.Wf, mfma_tile_w()) * cdiv(g.Hf, mfma_tile_h()));
  else
    pl.fwd_tiles = (int)(cdiv(g.Wf, fwd_tile_w(g)) * cdiv(g.Hf, fwd_tile_h(g)));
  int fg = (int)std::min<int64_t>(g.n, cdiv(target, pl.fwd_tiles));
  fg = std::max(fg, 1);
  pl.fwd_fpg = (int)cdiv(g.n, fg);
  if (uses_m2n(g)) pl.fwd_fpg = M2N_FPG;   // the frames are the products' N dimension
  pl.fwd_groups = (int)cdiv(g.n, pl.fwd_fpg);
  pl.adj_variant = 0;
  if (mf && g.sr == 2)
    pl.adj_tiles = (int)(cdiv(g.Wl, mfma2_adj_tile_w(g.precision)) *
                         cdiv(g.Hl, mfma2_adj_tile_h(g.precision)));
  else if (mf)
    pl.adj_tiles = (int)(cdiv(g.Wl, mfma_tile_w()) * cdiv(g.Hl, mfma_tile_h()));
  else
    pl.adj_tiles = (int)(cdiv(g.Wl, adj_tile_w(g)) * cdiv(g.Hl, adj_tile_h(g)));
  if (pl.adj_tiles >= (mf ? target / 4 : target / 2)) {
    pl.adj_groups = 1;
    pl.adj_fpg = g.n;
  } else {
    int ag = (int)std::min<int64_t>(g.n, cdiv(target, pl.adj_tiles));
    ag = std::max(ag, 1);
    pl.adj_fpg = (int)cdiv(g.n, ag);
    pl.adj_groups = (int)cdiv(g.n, pl.adj_fpg);
  }
  if (g.weight_mode == EM_W_LITERAL) {
    // the typeset weighting multiplies each frame's adjoint by its own u:
    // one frame per group, weighted sum of the planes afterwards
    pl.adj_fpg = 1;
    pl.adj_groups = g.n;
  }
  pl.adj_fused = pl.adj_groups == 1 && g.weight_mode != EM_W_LITERAL;
  // every job starts on the default variants; only em_autotune or
  // em_set_variants on that job change them
  pl.fwd_variant = 0;
  pl.adj_variant = 0;
  pl.prep_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, cdiv((int64_t)g.n * g.Nf, 256)));
  pl.upd_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(4096, cdiv(g.Nl, 256)));
  pl.max_partials = std::max(pl.fwd_tiles * pl.fwd_groups, std::max(pl.adj_tiles, pl.upd_blocks));
  return pl;
}

// Plan of a job run by the serving loop: the frame sum of the adjoint is never
// split (update fused, no partial planes), the forward uses groups of at most
// four frames (the grouping does not change its arithmetic), and the matrix-core
// kernels use fixed variants.  The plan depends on the job's shape only.
Plan make_serving_plan(const Geometry& g) {
  Plan pl = make_plan(g);
  pl.adj_groups = 1;
  pl.adj_fpg = g.n;
  pl.adj_fused = 1;
  if (!uses_m2n(g)) pl.fwd_fpg = std::min(g.n, 4);
  pl.fwd_groups = (int)cdiv(g.n, pl.fwd_fpg);
  pl.max_partials = std::max(pl.fwd_tiles * pl.fwd_groups, std::max(pl.adj_tiles, pl.upd_blocks));
  if (uses_mfma(g)) {
    // the variants em_autotune picks on the large workloads (33 x 4096^2 sr = 1,
    // 16 x 2048^2 sr = 2) for each encoding (the sr = 1 FP16 forward: 4x2 blocks
    // per wave with the image fragments loaded ahead; the sr = 2 forward of jobs
    // with its frames in the N dimension: 4 rows x 2 blocks per wave in the FP16
    // split form, 4 rows x 1 block in the BF16 split form); for the sr = 2 FP16
    // adjoint the 4x2-block variant, 3% slower alone but free of scratch reloads
    // in its batched form
    const bool f16 = g.precision == EM_FP16_SPLIT;
    pl.fwd_variant = g.sr == 1 ? (f16 ? 1 : 0) : (uses_m2n(g) ? (f16 ? 1 : 0) : (f16 ? 2 : 0));
    pl.adj_variant = g.sr == 1 ? 2 : (f16 ? 1 : 0);
  }
  return pl;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

Layout make_layout(const Geometry& g, const Plan& pl) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += al256(bytes);
    return o;
  };
  const size_t nf = (size_t)g.n * g.Nf;
  // frame groups for per-frame adjoint output of em_adjoint_op use the caller's buffer
  const int G = pl.adj_groups;
  L.u = take(nf * sizeof(float));
  L.r = take(nf * sizeof(float));
  L.ry = take(g.weight_mode == EM_W_STUDENT_T ? nf * sizeof(float) : 0);
  L.B = take((size_t)g.Nl * sizeof(float));
  L.planes = take(pl.adj_fused ? 0 : (size_t)G * g.Nl * sizeof(float));
  L.tab = take((size_t)g.n * g.KC * TAB_LD * sizeof(float));
  L.mtab_fwd = take(uses_mfma(g) ? mfma_table_bytes(g, 0) : 0);
  L.mtab_adj = take(uses_mfma(g) ? mfma_table_bytes(g, 1) : 0);
  L.tune = take(uses_mfma(g) ? (size_t)g.Nl * sizeof(float) : 0);
  L.part_ll = take((size_t)std::max(pl.fwd_tiles * pl.fwd_groups, pl.prep_blocks) * sizeof(double));
  L.part_rc = take((size_t)2 * std::max(pl.adj_tiles, pl.upd_blocks) * sizeof(double));
  L.part_prep = take((size_t)3 * pl.prep_blocks * sizeof(double));
  L.scalars = take(S_COUNT * sizeof(double));
  L.trace_ll = take(TRACE_CAP * sizeof(double));
  L.trace_rc = take(TRACE_CAP * sizeof(double));
  L.counters = take(16 * sizeof(int));
  const bool r16 = uses_r16(g);
  L.r16 = take(r16 ? (size_t)g.n * r16_rows(g) * r16_pitch(g) * sizeof(uint16_t) : 0);
  L.r16stat = take(r16 ? (size_t)(3 * g.n + R16_XBLOCKS) * sizeof(float) : 0);
  L.total = off;
  return L;
}

// Checks that [ptr, ptr + bytes) lies inside one device allocation.
static int check_device_range(const void* ptr, size_t bytes, const char* name) {
  if (ptr == nullptr) return fail(EM_EINVAL, "%s is NULL", name);
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(EM_EINVAL, "%s is not a HIP device pointer", name);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(EM_EINVAL, "%s is not device memory", name);
  void* base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(reinterpret_cast<hipDeviceptr_t*>(&base), &size,
                            reinterpret_cast<hipDeviceptr_t>(const_cast<void*>(ptr)));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(EM_EINVAL, "%s: cannot query the allocation", name);
  }
  const char* b = static_cast<const char*>(base);
  const char* p = static_cast<const char*>(ptr);
  if (p < b || p + bytes > b + size)
    return fail(EM_EINVAL, "%s: buffer smaller than the %zu bytes needed", name, bytes);
  return EM_OK;
}

}  // namespace em

using namespace em;

void em_bind_views(em_ctx* c) {
  char* w = c->ws;
  const Layout& L = c->lay;
  c->u = reinterpret_cast<float*>(w + L.u);
  c->r = reinterpret_cast<float*>(w + L.r);
  c->ry = reinterpret_cast<float*>(w + L.ry);
  c->B = reinterpret_cast<float*>(w + L.B);
  c->planes = reinterpret_cast<float*>(w + L.planes);
  c->tab = reinterpret_cast<float*>(w + L.tab);
  c->mtab_fwd = w + L.mtab_fwd;
  c->mtab_adj = w + L.mtab_adj;
  c->tune = reinterpret_cast<float*>(w + L.tune);
  c->part_ll = reinterpret_cast<double*>(w + L.part_ll);
  c->part_rc = reinterpret_cast<double*>(w + L.part_rc);
  c->part_prep = reinterpret_cast<double*>(w + L.part_prep);
  c->scalars = reinterpret_cast<double*>(w + L.scalars);
  c->trace_ll = reinterpret_cast<double*>(w + L.trace_ll);
  c->trace_rc = reinterpret_cast<double*>(w + L.trace_rc);
  c->counters = reinterpret_cast<int*>(w + L.counters);
  c->r16 = reinterpret_cast<unsigned short*>(w + L.r16);
  c->r16_umax = reinterpret_cast<float*>(w + L.r16stat);
  c->r16_fsum = c->r16_umax + c->g.n;
  c->r16_e = reinterpret_cast<int*>(c->r16_fsum + c->g.n);
  c->r16_xpart = reinterpret_cast<float*>(c->r16_e + c->g.n);
}

extern "C" {

const char* em_version(void) {
  return "libem 0.1 (gfx950; FP32 direct convolution; FP64 reductions)";
}

const char* em_last_error(void) { return em::g_last_error.c_str(); }

size_t em_workspace_bytes(const em_problem* p) {
  Geometry g;
  const char* why = nullptr;
  if (!make_geometry(p, &g, &why)) return 0;
  const Plan pl = make_plan(g);
  return make_layout(g, pl).total;
}

}  // extern "C"

// Adjoint of every frame of `in` (n x Nf), summed over frames, into `out`
// (Nl floats); never applies the update.
static int adjoint_sum(em_ctx* c, const float* in, float* out) {
  const bool lit = c->g.weight_mode == EM_W_LITERAL;
  const bool via_planes = c->pl.adj_groups > 1 || lit;
  float* dst = via_planes ? c->planes : out;
  if (uses_mfma(c->g)) {
    MfmaLaunch m{};
    m.in = in;
    m.tab = c->mtab_adj;
    m.plane = dst;
    m.n = c->g.n;
    m.H = c->g.Hl;
    m.W = c->g.Wl;
    m.fpg = c->pl.adj_fpg;
    m.ntiles = c->pl.adj_tiles;
    m.fused = 0;
    m.lo_band = c->pl.lo_band;
    EM_HIP(launch_mfma(c->g, 1, c->pl.adj_variant, c->pl.adj_tiles, c->pl.adj_groups, m,
                       c->stream));
  } else {
    AdjLaunch a{};
    a.in = in;
    a.tab = c->tab;
    a.n = c->g.n;
    a.Hf = c->g.Hf;
    a.Wf = c->g.Wf;
    a.Hl = c->g.Hl;
    a.Wl = c->g.Wl;
    a.fpg = c->pl.adj_fpg;
    a.ntiles = c->pl.adj_tiles;
    a.fused = 0;
    a.plane = dst;
    EM_HIP(launch_adjoint(c->g, c->pl, a, c->stream));
  }
  if (via_planes)
    EM_HIP(launch_sum_planes(c->planes, lit ? c->u : nullptr, c->pl.adj_groups, c->g.Nl, out,
                             c->stream));
  return EM_OK;
}

namespace em {

void fill_forward_mfma(const em_ctx* c, MfmaLaunch* m, bool write_r, bool loglik) {
  *m = MfmaLaunch{};
  m->in = c->x;
  m->tab = c->mtab_fwd;
  m->u = c->u;
  m->y = c->y;
  m->out = write_r ? c->r : nullptr;
  m->part = loglik ? c->part_ll : nullptr;
  m->n = c->g.n;
  m->H = c->g.Hf;
  m->W = c->g.Wf;
  m->fpg = c->pl.fwd_fpg;
  m->ntiles = c->pl.fwd_tiles;
  m->lo_band = c->pl.lo_band;
}

void fill_forward_fp32(const em_ctx* c, FwdLaunch* f, bool write_r, bool loglik) {
  *f = FwdLaunch{};
  f->x = c->x;
  f->tab = c->tab;
  f->u = c->u;
  f->y = c->y;
  f->out = write_r ? c->r : nullptr;
  f->part = loglik ? c->part_ll : nullptr;
  f->n = c->g.n;
  f->Hf = c->g.Hf;
  f->Wf = c->g.Wf;
  f->Hl = c->g.Hl;
  f->Wl = c->g.Wl;
  f->fpg = c->pl.fwd_fpg;
  f->ntiles = c->pl.fwd_tiles;
}

void fill_adjoint_mfma(const em_ctx* c, MfmaLaunch* m, double* part_rc) {
  const bool fused = c->pl.adj_fused != 0;
  *m = MfmaLaunch{};
  m->in = c->r;
  m->tab = c->mtab_adj;
  m->n = c->g.n;
  m->H = c->g.Hl;
  m->W = c->g.Wl;
  m->fpg = c->pl.adj_fpg;
  m->ntiles = c->pl.adj_tiles;
  m->fused = fused ? 1 : 0;
  m->x = c->x;
  m->B = c->B;
  m->part = fused ? part_rc : nullptr;
  m->plane = c->planes;
  m->lo_band = c->pl.lo_band;
}

void fill_adjoint_fp32(const em_ctx* c, AdjLaunch* a, double* part_rc) {
  const bool fused = c->pl.adj_fused != 0;
  *a = AdjLaunch{};
  a->in = c->r;
  a->tab = c->tab;
  a->n = c->g.n;
  a->Hf = c->g.Hf;
  a->Wf = c->g.Wf;
  a->Hl = c->g.Hl;
  a->Wl = c->g.Wl;
  a->fpg = c->pl.adj_fpg;
  a->ntiles = c->pl.adj_tiles;
  a->fused = fused ? 1 : 0;
  a->x = c->x;
  a->B = c->B;
  a->part = fused ? part_rc : nullptr;
  a->plane = c->planes;
}

// The iteration of an FP16 split sr = 1 job with Gaussian weights moves r
// through binary16 planes: the forward writes them, the adjoint copies its
// windows from them (dir 0: forward descriptor; dir 1: adjoint descriptor).
void apply_r16(const em_ctx* c, MfmaLaunch* m, int dir) {
  m->r16 = c->r16;
  m->e16 = c->r16_e;
  m->p16 = r16_pitch(c->g);
  m->s16 = (int64_t)r16_rows(c->g) * r16_pitch(c->g);
  if (dir == 0) m->out = nullptr;
  else m->in = nullptr;
}

}  // namespace em

static int r16_scale(em_ctx* c) {
  EM_HIP(launch_r16_scale(c->g, c->x, c->r16_xpart, c->r16_umax, c->r16_fsum, c->r16_e,
                          c->stream));
  return EM_OK;
}

// Forward pass at the current iterate: r = u F x (if write_r) and loglik
// partials.  Under the typeset weighting r is the raw model F x (the weights act
// after the adjoint) and the loglik partials come from a separate pass over r,
// u and y.  *n_ll: the number of loglik partials written (may be NULL).
// With r16 (the iteration of an FP16 split job, uses_r16) r goes to the
// binary16 planes, whose scales r16_scale has set.
static int forward_pass(em_ctx* c, bool write_r, bool loglik, int* n_ll = nullptr,
                        bool r16 = false) {
  const bool raw = write_r && c->g.weight_mode == EM_W_LITERAL;
  if (n_ll) *n_ll = c->pl.fwd_tiles * c->pl.fwd_groups;
  if (uses_mfma(c->g)) {
    MfmaLaunch m;
    fill_forward_mfma(c, &m, write_r, loglik && !raw);
    if (raw) m.u = nullptr;
    if (r16 && write_r) apply_r16(c, &m, 0);
    EM_HIP(launch_mfma(c->g, 0, c->pl.fwd_variant, c->pl.fwd_tiles, c->pl.fwd_groups, m,
                       c->stream));
  } else {
    FwdLaunch f;
    fill_forward_fp32(c, &f, write_r, loglik && !raw);
    if (raw) f.u = nullptr;
    EM_HIP(launch_forward(c->g, c->pl, f, c->stream));
  }
  if (raw && loglik) {
    EM_HIP(launch_loglik_partials(c->r, c->u, c->y, (int64_t)c->g.n * c->g.Nf, c->part_ll,
                                  c->pl.prep_blocks, c->stream));
    if (n_ll) *n_ll = c->pl.prep_blocks;
  }
  return EM_OK;
}

// Student-t noise: the forward epilogue applies the E-step weights, writing
// r = u w F x and ry = u w y, with Student-t loglik partials when asked.
double em::student_t_lcst(double nu) {
  return 2.0 * (std::lgamma(0.5 * (nu + 1.0)) - std::lgamma(0.5 * nu) - 0.5 * std::log(nu * M_PI)) +
         std::log(2.0 * M_PI);
}

static int robust_forward(em_ctx* c, bool loglik) {
  const double lcst = student_t_lcst((double)c->g.nu);
  if (uses_mfma(c->g)) {
    MfmaLaunch m;
    fill_forward_mfma(c, &m, true, loglik);
    m.out_y = c->ry;
    m.nu = c->g.nu;
    m.lcst = lcst;
    EM_HIP(launch_mfma(c->g, 0, c->pl.fwd_variant, c->pl.fwd_tiles, c->pl.fwd_groups, m,
                       c->stream));
  } else {
    FwdLaunch f;
    fill_forward_fp32(c, &f, true, loglik);
    f.out_y = c->ry;
    f.nu = c->g.nu;
    f.lcst = lcst;
    EM_HIP(launch_forward(c->g, c->pl, f, c->stream));
  }
  return EM_OK;
}

// Adjoint of r summed over frames; with a single frame group the
// multiplicative update is fused into its epilogue, else it writes the partial
// planes (the update then runs separately, update_launch).
static int adjoint_launch(em_ctx* c, double* part_rc) {
  if (uses_mfma(c->g)) {
    MfmaLaunch m;
    fill_adjoint_mfma(c, &m, part_rc);
    if (uses_r16(c->g)) apply_r16(c, &m, 1);
    EM_HIP(launch_mfma(c->g, 1, c->pl.adj_variant, c->pl.adj_tiles, c->pl.adj_groups, m,
                       c->stream));
  } else {
    AdjLaunch a;
    fill_adjoint_fp32(c, &a, part_rc);
    EM_HIP(launch_adjoint(c->g, c->pl, a, c->stream));
  }
  return EM_OK;
}

static int update_launch(em_ctx* c, double* part_rc) {
  const float* w = c->g.weight_mode == EM_W_LITERAL ? c->u : nullptr;
  EM_HIP(launch_update(c->planes, w, c->pl.adj_groups, c->g.Nl, c->B, c->x, part_rc,
                       c->pl.upd_blocks, c->stream));
  return EM_OK;
}

// Adjoint + update; *n_rc = number of change partials written.
static int adjoint_update(em_ctx* c, double* part_rc, int* n_rc) {
  int rc = adjoint_launch(c, part_rc);
  if (rc) return rc;
  if (c->pl.adj_fused) {
    *n_rc = c->pl.adj_tiles;
    return EM_OK;
  }
  *n_rc = c->pl.upd_blocks;
  return update_launch(c, part_rc);
}

// One EM iteration (Eq. (2)); optional FP64 loglik / relative-change bookkeeping.
// Under Student-t noise the numerator is formed again from the new weights
// before the adjoint of the denominator (which applies the update).
static int one_iteration(em_ctx* c, bool loglik, bool relchange) {
  const bool robust = c->g.weight_mode == EM_W_STUDENT_T;
  int n_ll = c->pl.fwd_tiles * c->pl.fwd_groups;
  const bool r16 = uses_r16(c->g);
  int rc = r16 ? r16_scale(c) : EM_OK;
  if (rc) return rc;
  rc = robust ? robust_forward(c, loglik) : forward_pass(c, true, loglik, &n_ll, r16);
  if (rc) return rc;
  if (robust && (rc = adjoint_sum(c, c->ry, c->B))) return rc;
  int n_rc = 0;
  if ((rc = adjoint_update(c, relchange ? c->part_rc : nullptr, &n_rc))) return rc;
  if (loglik || relchange) {
    EM_HIP(launch_finalize_iter(loglik ? c->part_ll : nullptr, n_ll,
                                relchange ? c->part_rc : nullptr, n_rc, c->scalars, c->trace_ll,
                                c->trace_rc, c->counters, c->stream));
  }
  return EM_OK;
}


static void drop_graphs(em_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->graph_ok[k]) (void)hipGraphExecDestroy(c->graph[k]);
    c->graph_ok[k] = false;
  }
}

// n iterations; when the job's stream is a created stream (graph capture is not
// available on the legacy default stream) one iteration is captured once into
// a HIP graph and replayed.  The captured iteration holds kernels only.
static int run_iterations(em_ctx* c, int n, bool loglik) {
  if (n <= 0) return EM_OK;
  const int k = loglik ? 1 : 0;
  if (c->stream != nullptr && !c->no_graph && !c->graph_ok[k]) {
    hipGraph_t gr = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const int rc = one_iteration(c, loglik, false);
      const hipError_t e = hipStreamEndCapture(c->stream, &gr);
      if (rc != EM_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
      }
      if (e == hipSuccess && gr != nullptr &&
          hipGraphInstantiate(&c->graph[k], gr, nullptr, nullptr, 0) == hipSuccess)
        c->graph_ok[k] = true;
      if (gr) (void)hipGraphDestroy(gr);
    }
    (void)hipGetLastError();
  }
  if (c->graph_ok[k]) {
    for (int i = 0; i < n; ++i) EM_HIP(hipGraphLaunch(c->graph[k], c->stream));
    return EM_OK;
  }
  for (int i = 0; i < n; ++i) {
    const int rc = one_iteration(c, loglik, false);
    if (rc) return rc;
  }
  return EM_OK;
}

extern "C" {

}  // extern "C"

// The checks and the device work of em_init on a context the caller provides
// (allocates nothing): u, yhat, the coefficient tables, B and x^(0) on the
// stream, which is synchronised to read the validation flags.  With
// check_workspace false the workspace is the library's own static scratch,
// which the caller has already sized.
static int setup_job(em_ctx* c, const em_problem* p, const float* y, const float* v,
                     const float* psf, const float* x0, float* x, void* workspace,
                     size_t ws_bytes, void* stream, bool serving, bool check_workspace) {
  Geometry g;
  const char* why = nullptr;
  if (!make_geometry(p, &g, &why)) return fail(EM_EINVAL, "invalid problem: %s", why);
  if (g.weight_mode == EM_W_LITERAL && g.sr != 1)
    return fail(EM_ENOTSUP, "the typeset weighting is defined for sr = 1 only");
  const Plan pl = serving ? make_serving_plan(g) : make_plan(g);
  const Layout L = make_layout(g, pl);
  if (ws_bytes < L.total)
    return fail(EM_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(EM_EINVAL, "workspace must be 256-byte aligned");
  const size_t fbytes = (size_t)g.n * g.Nf * sizeof(float);
  const size_t lbytes = (size_t)g.Nl * sizeof(float);
  int rc;
  if ((rc = check_device_range(y, fbytes, "y"))) return rc;
  if ((rc = check_device_range(v, fbytes, "v"))) return rc;
  if ((rc = check_device_range(psf, (size_t)g.n * g.K * g.K * sizeof(float), "psf"))) return rc;
  if (x0 && (rc = check_device_range(x0, lbytes, "x0"))) return rc;
  if ((rc = check_device_range(x, lbytes, "x"))) return rc;
  if (check_workspace && (rc = check_device_range(workspace, L.total, "workspace"))) return rc;

  c->g = g;
  c->pl = pl;
  c->lay = L;
  c->stream = static_cast<hipStream_t>(stream);
  c->y = y;
  c->v = v;
  c->psf = psf;
  c->x = x;
  c->ws = static_cast<char*>(workspace);
  em_bind_views(c);

  hipError_t e;
  if ((e = launch_reset_counters(c->counters, c->stream)) != hipSuccess ||
      (e = launch_reset_counters(c->counters + 4, c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "reset: %s", hipGetErrorString(e));
  PrepLaunch pr{};
  pr.y = y;
  pr.v = v;
  pr.u = c->u;
  pr.w = c->r;
  pr.part = c->part_prep;
  pr.flags = c->counters + 4;
  pr.count = (int64_t)g.n * g.Nf;
  pr.blocks = pl.prep_blocks;
  pr.raw_y = g.weight_mode == EM_W_LITERAL ? 1 : 0;
  if ((e = launch_prep(pr, c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "prep: %s", hipGetErrorString(e));
  if ((e = launch_psf_tables(g, psf, c->tab, c->counters + 4, c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "psf tables: %s", hipGetErrorString(e));
  if (uses_mfma(g) &&
      (e = launch_mfma_tables(g, psf, c->mtab_fwd, c->mtab_adj, c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "mfma tables: %s", hipGetErrorString(e));
  if (uses_r16(g) && (e = launch_r16_setup(g, c->u, psf, c->r16, c->r16_umax, c->r16_fsum,
                                           c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "r16 planes: %s", hipGetErrorString(e));
  // BF16 split (sr = 1, K = 43, not served): the lo band when every frame's PSF
  // keeps at most 1/16 of its mass outside it
  c->pl.lo_band = 0;
  if (!serving && g.precision == EM_BF16_SPLIT && g.sr == 1 && g.KT == KT_LARGE) {
    int over = 1;
    if ((e = launch_lo_band_check(g, psf, c->counters + 7, c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(&over, c->counters + 7, sizeof(int), hipMemcpyDeviceToHost,
                            c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
      return fail(EM_EDEVICE, "band check: %s", hipGetErrorString(e));
    c->pl.lo_band = over == 0 ? 1 : 0;
  }
  if ((rc = adjoint_sum(c, c->r, c->B))) return rc;
  if ((e = launch_finalize_prep(c->part_prep, pl.prep_blocks, c->scalars, g.sr, c->stream)) !=
      hipSuccess)
    return fail(EM_EDEVICE, "finalize: %s", hipGetErrorString(e));
  if ((e = launch_init_x(x0, x, c->scalars, g.Nl, c->counters + 4, c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "init x: %s", hipGetErrorString(e));
  int flags[4] = {0, 0, 0, 0};
  if ((e = hipMemcpyAsync(flags, c->counters + 4, sizeof(flags), hipMemcpyDeviceToHost,
                          c->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess)
    return fail(EM_EDEVICE, "init sync: %s", hipGetErrorString(e));
  if (flags[0]) return fail(EM_EINVAL, "%d invalid exposure/variance pixels", flags[0]);
  if (flags[1]) return fail(EM_EINVAL, "%d invalid PSF taps (must be finite, >= 0)", flags[1]);
  if (flags[2]) return fail(EM_EINVAL, "%d invalid x0 pixels (must be finite, >= 0)", flags[2]);
  return EM_OK;
}

int em::init_ctx(em_ctx** out, const em_problem* p, const float* y, const float* v,
                 const float* psf, const float* x0, float* x, void* workspace, size_t ws_bytes,
                 void* stream, bool serving) {
  if (!out) return fail(EM_EINVAL, "out is NULL");
  *out = nullptr;
  em_ctx* c = new (std::nothrow) em_ctx();
  if (!c) return fail(EM_ENOMEM, "host allocation failed");
  const int rc = setup_job(c, p, y, v, psf, x0, x, workspace, ws_bytes, stream, serving, true);
  if (rc != EM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return EM_OK;
}

extern "C" {

int em_init(em_ctx** out, const em_problem* p, const float* y, const float* v, const float* psf,
            const float* x0, float* x, void* workspace, size_t ws_bytes, void* stream) {
  return init_ctx(out, p, y, v, psf, x0, x, workspace, ws_bytes, stream, false);
}

int em_iterate(em_ctx* c, int32_t n_iter, double* loglik_trace) {
  if (!c) return fail(EM_EINVAL, "ctx is NULL");
  if (n_iter < 0) return fail(EM_EINVAL, "n_iter < 0");
  const bool tr = loglik_trace != nullptr;
  int done = 0;
  while (done < n_iter) {
    const int chunk = std::min(n_iter - done, TRACE_CAP);
    if (tr) EM_HIP(launch_reset_counters(c->counters, c->stream));
    int rc = run_iterations(c, chunk, tr);
    if (rc) return rc;
    if (tr) {
      EM_HIP(hipMemcpyAsync(loglik_trace + done, c->trace_ll, sizeof(double) * chunk,
                            hipMemcpyDeviceToHost, c->stream));
      EM_HIP(hipStreamSynchronize(c->stream));
    }
    done += chunk;
  }
  return EM_OK;
}

int em_iterate_tol(em_ctx* c, int32_t max_iter, double tol, int32_t check_every,
                   int32_t* iters_done, double* loglik_trace, double* relchange_trace) {
  if (!c) return fail(EM_EINVAL, "ctx is NULL");
  if (max_iter < 0 || check_every < 1) return fail(EM_EINVAL, "bad max_iter / check_every");
  if (!iters_done) return fail(EM_EINVAL, "iters_done is NULL");
  const bool tr = loglik_trace != nullptr;
  int done = 0;
  std::vector<double> rcbuf;
  while (done < max_iter) {
    const int chunk = std::min(std::min(max_iter - done, check_every), TRACE_CAP);
    EM_HIP(launch_reset_counters(c->counters, c->stream));
    for (int k = 0; k < chunk; ++k) {
      int rc = one_iteration(c, tr, true);
      if (rc) return rc;
    }
    rcbuf.resize(chunk);
    EM_HIP(hipMemcpyAsync(rcbuf.data(), c->trace_rc, sizeof(double) * chunk,
                          hipMemcpyDeviceToHost, c->stream));
    if (tr)
      EM_HIP(hipMemcpyAsync(loglik_trace + done, c->trace_ll, sizeof(double) * chunk,
                            hipMemcpyDeviceToHost, c->stream));
    EM_HIP(hipStreamSynchronize(c->stream));
    if (relchange_trace) std::copy(rcbuf.begin(), rcbuf.end(), relchange_trace + done);
    done += chunk;
    bool stop = false;
    for (int k = 0; k < chunk; ++k) stop = stop || rcbuf[k] < tol;
    if (stop) break;
  }
  *iters_done = done;
  return EM_OK;
}

int em_loglik(em_ctx* c, double* out) {
  if (!c || !out) return fail(EM_EINVAL, "NULL argument");
  int rc = c->g.weight_mode == EM_W_STUDENT_T ? robust_forward(c, true)
                                              : forward_pass(c, false, true);
  if (rc) return rc;
  EM_HIP(launch_finalize_loglik(c->part_ll, c->pl.fwd_tiles * c->pl.fwd_groups, c->scalars,
                                c->stream));
  EM_HIP(hipMemcpyAsync(out, c->scalars + S_LOGLIK, sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
  EM_HIP(hipStreamSynchronize(c->stream));
  return EM_OK;
}

int em_terms(em_ctx* c, float* B_out, float* Dn_out) {
  if (!c) return fail(EM_EINVAL, "ctx is NULL");
  const size_t lbytes = (size_t)c->g.Nl * sizeof(float);
  int rc;
  if (c->g.weight_mode == EM_W_STUDENT_T) {
    // both terms depend on the weights at the current iterate
    if (B_out && (rc = check_device_range(B_out, lbytes, "B_out"))) return rc;
    if (Dn_out && (rc = check_device_range(Dn_out, lbytes, "Dn_out"))) return rc;
    if ((rc = robust_forward(c, false))) return rc;
    if (B_out && (rc = adjoint_sum(c, c->ry, B_out))) return rc;
    if (Dn_out && (rc = adjoint_sum(c, c->r, Dn_out))) return rc;
    return EM_OK;
  }
  if (B_out) {
    if ((rc = check_device_range(B_out, lbytes, "B_out"))) return rc;
    EM_HIP(hipMemcpyAsync(B_out, c->B, lbytes, hipMemcpyDeviceToDevice, c->stream));
  }
  if (Dn_out) {
    if ((rc = check_device_range(Dn_out, lbytes, "Dn_out"))) return rc;
    if ((rc = forward_pass(c, true, false))) return rc;
    if ((rc = adjoint_sum(c, c->r, Dn_out))) return rc;
  }
  return EM_OK;
}

int em_profile(em_ctx* c, int32_t n_iter, double* phase_ms) {
  if (!c || !phase_ms) return fail(EM_EINVAL, "NULL argument");
  if (n_iter < 1) return fail(EM_EINVAL, "n_iter must be >= 1");
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) EM_HIP(hipEventCreate(&ev[i]));
  const bool r16 = uses_r16(c->g);
  double acc[4] = {0, 0, 0, 0};
  int rc = EM_OK;
  const bool fused = c->pl.adj_fused != 0;
  const bool robust = c->g.weight_mode == EM_W_STUDENT_T;
  for (int k = 0; k < n_iter && rc == EM_OK; ++k) {
    EM_HIP(hipEventRecord(ev[0], c->stream));
    if (r16 && (rc = r16_scale(c))) break;
    EM_HIP(hipEventRecord(ev[5], c->stream));
    if ((rc = robust ? robust_forward(c, false) : forward_pass(c, true, false, nullptr, r16))) break;
    EM_HIP(hipEventRecord(ev[4], c->stream));
    if (robust && (rc = adjoint_sum(c, c->ry, c->B))) break;
    EM_HIP(hipEventRecord(ev[1], c->stream));
    if ((rc = adjoint_launch(c, nullptr))) break;
    EM_HIP(hipEventRecord(ev[2], c->stream));
    if (!fused && (rc = update_launch(c, nullptr))) break;
    EM_HIP(hipEventRecord(ev[3], c->stream));
    EM_HIP(hipEventSynchronize(ev[3]));
    float ms;
    EM_HIP(hipEventElapsedTime(&ms, ev[5], ev[4]));
    acc[0] += ms;
    EM_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
    acc[1] += ms;
    EM_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
    acc[2] += fused ? 0.0 : ms;
    EM_HIP(hipEventElapsedTime(&ms, ev[0], ev[3]));
    acc[3] += ms;
  }
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  if (rc) return rc;
  for (int i = 0; i < 4; ++i) phase_ms[i] = acc[i] / n_iter;
  return EM_OK;
}

int em_check_plan(const em_problem* p) {
  Geometry g;
  const char* why = nullptr;
  if (!make_geometry(p, &g, &why)) return fail(EM_EINVAL, "invalid problem: %s", why);
  for (int serving = 0; serving < 2; ++serving) {
    const Plan pl = serving ? make_serving_plan(g) : make_plan(g);
    em_ctx c{};
    c.g = g;
    c.pl = pl;
    c.lay = make_layout(g, pl);
    c.ws = reinterpret_cast<char*>(static_cast<uintptr_t>(1) << 20);   // never dereferenced
    em_bind_views(&c);
    const char* what = serving ? "serving plan" : "plan";
    for (int v = 0; v < (uses_mfma(g) ? mfma_variants() : 1); ++v) {
      c.pl.fwd_variant = c.pl.adj_variant = v;
      if (uses_mfma(g)) {
        MfmaLaunch m;
        fill_forward_mfma(&c, &m, true, true);
        if (!mfma_desc_ok(g, 0, pl.fwd_tiles, pl.fwd_groups, m))
          return fail(EM_EINVAL, "%s: forward descriptor does not match its grid", what);
        fill_adjoint_mfma(&c, &m, nullptr);
        if (!mfma_desc_ok(g, 1, pl.adj_tiles, pl.adj_groups, m))
          return fail(EM_EINVAL, "%s: adjoint descriptor does not match its grid", what);
        if (uses_r16(g) && !serving) {
          // the iteration's binary16 r planes
          MfmaLaunch f16;
          fill_forward_mfma(&c, &f16, true, true);
          apply_r16(&c, &f16, 0);
          if (!mfma_desc_ok(g, 0, pl.fwd_tiles, pl.fwd_groups, f16))
            return fail(EM_EINVAL, "%s: r16 forward descriptor does not match", what);
          MfmaLaunch a16 = m;
          apply_r16(&c, &a16, 1);
          if (!mfma_desc_ok(g, 1, pl.adj_tiles, pl.adj_groups, a16))
            return fail(EM_EINVAL, "%s: r16 adjoint descriptor does not match", what);
          // every window of every tile, and every pixel the forward writes,
          // inside its plane
          int64_t last_row, last_col;
          if (g.sr == 2) {
            const int th = mfma2_adj_tile_h(EM_FP16_SPLIT), tw = mfma2_adj_tile_w(EM_FP16_SPLIT);
            last_row = (int64_t)((g.Hl + th - 1) / th - 1) * (th / 2) + th / 2 + 31;
            last_col = (int64_t)((g.Wl + tw - 1) / tw - 1) * (tw / 2) + tw / 2 + 47;
          } else {
            last_row = (int64_t)((g.Hl + 127) / 128 - 1) * 128 + 127 + g.KT - 1;
            last_col = (int64_t)((g.Wl + 127) / 128 - 1) * 128 + 175;
          }
          if (last_row >= r16_rows(g) || last_col >= r16_pitch(g) || r16_pitch(g) % 8 != 0 ||
              g.Hf - 1 + r16_off(g) >= r16_rows(g) || g.Wf - 1 + r16_off(g) >= r16_pitch(g) ||
              c.lay.r16stat - c.lay.r16 < (size_t)g.n * r16_rows(g) * r16_pitch(g) * 2)
            return fail(EM_EINVAL, "%s: r16 planes smaller than the windows", what);
        }
        m.fpg = 1;   // stand-alone operator: one frame per group
        if (!mfma_desc_ok(g, 1, pl.adj_tiles, g.n, m))
          return fail(EM_EINVAL, "%s: per-frame adjoint descriptor does not match", what);
      } else {
        FwdLaunch f;
        fill_forward_fp32(&c, &f, true, true);
        if (!forward_desc_ok(g, pl.fwd_tiles, pl.fwd_groups, f))
          return fail(EM_EINVAL, "%s: forward descriptor does not match its grid", what);
        AdjLaunch a;
        fill_adjoint_fp32(&c, &a, nullptr);
        if (!adjoint_desc_ok(g, pl.adj_tiles, pl.adj_groups, a))
          return fail(EM_EINVAL, "%s: adjoint descriptor does not match its grid", what);
        a.fpg = 1;
        if (!adjoint_desc_ok(g, pl.adj_tiles, g.n, a))
          return fail(EM_EINVAL, "%s: per-frame adjoint descriptor does not match", what);
      }
    }
    // workspace capacities for what the kernels write
    const Layout& L = c.lay;
    const size_t ll = (size_t)std::max(pl.fwd_tiles * pl.fwd_groups, pl.prep_blocks) * sizeof(double);
    const size_t rcb = (size_t)2 * std::max(pl.adj_tiles, pl.upd_blocks) * sizeof(double);
    if (L.part_rc - L.part_ll < ll || L.part_prep - L.part_rc < rcb)
      return fail(EM_EINVAL, "%s: partial-sum buffers too small", what);
    if (!pl.adj_fused && L.tab - L.planes < (size_t)pl.adj_groups * g.Nl * sizeof(float))
      return fail(EM_EINVAL, "%s: partial planes too small", what);
  }
  return EM_OK;
}

int em_variant_count(void) { return mfma_variants(); }

int em_set_variants(em_ctx* c, int32_t fwd_variant, int32_t adj_variant) {
  if (!c) return fail(EM_EINVAL, "ctx is NULL");
  if (!uses_mfma(c->g)) return fail(EM_ENOTSUP, "variants exist for matrix-core precisions only");
  if (fwd_variant < 0 || fwd_variant >= mfma_variants() || adj_variant < 0 ||
      adj_variant >= mfma_variants())
    return fail(EM_EINVAL, "variant out of range");
  c->pl.fwd_variant = fwd_variant;
  c->pl.adj_variant = adj_variant;
  drop_graphs(c);
  return EM_OK;
}

int em_autotune(em_ctx* c, int32_t n_rep, int32_t* fwd_variant, int32_t* adj_variant,
                double* ms) {
  if (!c) return fail(EM_EINVAL, "ctx is NULL");
  if (!uses_mfma(c->g)) return fail(EM_ENOTSUP, "variants exist for matrix-core precisions only");
  if (n_rep < 1) return fail(EM_EINVAL, "n_rep must be >= 1");
  const int nv = mfma_variants();
  hipEvent_t e0, e1;
  EM_HIP(hipEventCreate(&e0));
  EM_HIP(hipEventCreate(&e1));
  std::vector<double> t(2 * nv, 0.0);
  int rc = EM_OK;
  for (int dir = 0; dir < 2 && rc == EM_OK; ++dir) {
    for (int v = 0; v < nv && rc == EM_OK; ++v) {
      // descriptors of the iteration itself (grid sizes of the right grids)
      MfmaLaunch m;
      int tiles, groups;
      if (dir == 0) {
        // the forward writes r (and u w y under Student-t noise), which every
        // iteration recomputes before use
        fill_forward_mfma(c, &m, true, false);
        if (c->g.weight_mode == EM_W_STUDENT_T) {
          m.out_y = c->ry;
          m.nu = c->g.nu;
          m.lcst = student_t_lcst((double)c->g.nu);
        }
        if (uses_r16(c->g)) {
          apply_r16(c, &m, 0);
          if ((rc = r16_scale(c))) break;
        }
        tiles = c->pl.fwd_tiles;
        groups = c->pl.fwd_groups;
      } else {
        // the adjoint writes partial planes (never the iterate)
        fill_adjoint_mfma(c, &m, nullptr);
        if (uses_r16(c->g)) apply_r16(c, &m, 1);
        m.fused = 0;
        m.plane = c->pl.adj_groups > 1 ? c->planes : c->tune;
        tiles = c->pl.adj_tiles;
        groups = c->pl.adj_groups;
      }
      for (int k = 0; k <= n_rep && rc == EM_OK; ++k) {
        if (k == 1) EM_HIP(hipEventRecord(e0, c->stream));
        hipError_t e = launch_mfma(c->g, dir, v, tiles, groups, m, c->stream);
        if (e != hipSuccess) rc = fail(EM_EDEVICE, "autotune launch: %s", hipGetErrorString(e));
      }
      if (rc) break;
      EM_HIP(hipEventRecord(e1, c->stream));
      EM_HIP(hipEventSynchronize(e1));
      float el = 0.f;
      EM_HIP(hipEventElapsedTime(&el, e0, e1));
      t[dir * nv + v] = el / n_rep;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  int bf = 0, ba = 0;
  for (int v = 1; v < nv; ++v) {
    if (t[v] < t[bf]) bf = v;
    if (t[nv + v] < t[nv + ba]) ba = v;
  }
  c->pl.fwd_variant = bf;
  c->pl.adj_variant = ba;
  drop_graphs(c);
  if (fwd_variant) *fwd_variant = bf;
  if (adj_variant) *adj_variant = ba;
  if (ms) std::copy(t.begin(), t.end(), ms);
  return EM_OK;
}

int em_sync(em_ctx* c) {
  if (!c) return fail(EM_EINVAL, "ctx is NULL");
  EM_HIP(hipStreamSynchronize(c->stream));
  return EM_OK;
}

int em_destroy(em_ctx* c) {
  if (c) drop_graphs(c);
  delete c;
  return EM_OK;
}

// ---- stand-alone operators -------------------------------------------------

static int op_setup(const em_problem* p, const float* psf, void* workspace, size_t ws_bytes,
                    Geometry* g, Plan* pl, Layout* L) {
  const char* why = nullptr;
  if (!make_geometry(p, g, &why)) return fail(EM_EINVAL, "invalid problem: %s", why);
  *pl = make_plan(*g);
  *L = make_layout(*g, *pl);
  if (ws_bytes < L->total) return fail(EM_ENOMEM, "workspace too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(EM_EINVAL, "workspace must be 256-byte aligned");
  int rc;
  if ((rc = check_device_range(workspace, L->total, "workspace"))) return rc;
  if ((rc = check_device_range(psf, (size_t)g->n * g->K * g->K * sizeof(float), "psf"))) return rc;
  return EM_OK;
}

int em_forward_op(const em_problem* p, const float* psf, const float* x, float* m, void* workspace,
                  size_t ws_bytes, void* stream) {
  Geometry g;
  Plan pl;
  Layout L;
  int rc = op_setup(p, psf, workspace, ws_bytes, &g, &pl, &L);
  if (rc) return rc;
  if ((rc = check_device_range(x, (size_t)g.Nl * sizeof(float), "x"))) return rc;
  if ((rc = check_device_range(m, (size_t)g.n * g.Nf * sizeof(float), "m"))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  float* tab = reinterpret_cast<float*>(w + L.tab);
  int* flags = reinterpret_cast<int*>(w + L.counters);
  EM_HIP(launch_reset_counters(flags, s));
  EM_HIP(launch_psf_tables(g, psf, tab, flags, s));
  if (uses_mfma(g)) {
    EM_HIP(launch_mfma_tables(g, psf, w + L.mtab_fwd, w + L.mtab_adj, s));
    MfmaLaunch mm{};
    mm.in = x;
    mm.tab = w + L.mtab_fwd;
    mm.out = m;
    mm.n = g.n;
    mm.H = g.Hf;
    mm.W = g.Wf;
    mm.fpg = pl.fwd_fpg;
    mm.ntiles = pl.fwd_tiles;
    EM_HIP(launch_mfma(g, 0, pl.fwd_variant, pl.fwd_tiles, pl.fwd_groups, mm, s));
    return EM_OK;
  }
  FwdLaunch f{};
  f.x = x;
  f.tab = tab;
  f.u = nullptr;
  f.y = nullptr;
  f.out = m;
  f.part = nullptr;
  f.n = g.n;
  f.Hf = g.Hf;
  f.Wf = g.Wf;
  f.Hl = g.Hl;
  f.Wl = g.Wl;
  f.fpg = pl.fwd_fpg;
  f.ntiles = pl.fwd_tiles;
  EM_HIP(launch_forward(g, pl, f, s));
  return EM_OK;
}

int em_adjoint_op(const em_problem* p, const float* psf, const float* r, float* sout,
                  void* workspace, size_t ws_bytes, void* stream) {
  Geometry g;
  Plan pl;
  Layout L;
  int rc = op_setup(p, psf, workspace, ws_bytes, &g, &pl, &L);
  if (rc) return rc;
  if ((rc = check_device_range(r, (size_t)g.n * g.Nf * sizeof(float), "r"))) return rc;
  if ((rc = check_device_range(sout, (size_t)g.n * g.Nl * sizeof(float), "s"))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  float* tab = reinterpret_cast<float*>(w + L.tab);
  int* flags = reinterpret_cast<int*>(w + L.counters);
  EM_HIP(launch_reset_counters(flags, s));
  EM_HIP(launch_psf_tables(g, psf, tab, flags, s));
  Plan per = pl;  // one frame per group: group t writes plane t = F_t^T r_t
  per.adj_fpg = 1;
  per.adj_groups = g.n;
  if (uses_mfma(g)) {
    EM_HIP(launch_mfma_tables(g, psf, w + L.mtab_fwd, w + L.mtab_adj, s));
    MfmaLaunch mm{};
    mm.in = r;
    mm.tab = w + L.mtab_adj;
    mm.plane = sout;
    mm.n = g.n;
    mm.H = g.Hl;
    mm.W = g.Wl;
    mm.fpg = 1;
    mm.ntiles = pl.adj_tiles;
    mm.fused = 0;
    EM_HIP(launch_mfma(g, 1, pl.adj_variant, pl.adj_tiles, g.n, mm, s));
    return EM_OK;
  }
  AdjLaunch a{};
  a.in = r;
  a.tab = tab;
  a.plane = sout;
  a.n = g.n;
  a.Hf = g.Hf;
  a.Wf = g.Wf;
  a.Hl = g.Hl;
  a.Wl = g.Wl;
  a.fpg = 1;
  a.fused = 0;
  a.ntiles = pl.adj_tiles;
  EM_HIP(launch_adjoint(g, per, a, s));
  return EM_OK;
}

int em_upsample(int32_t n_frames, int32_t frame_h, int32_t frame_w, int32_t factor,
                const float* y, const float* v, float* y_up, float* v_up, void* stream) {
  if (n_frames < 1 || frame_h < 1 || frame_w < 1) return fail(EM_EINVAL, "sizes must be >= 1");
  if (factor < 2 || factor > 4) return fail(EM_EINVAL, "factor must be 2, 3 or 4");
  const int64_t nf = (int64_t)n_frames * frame_h * frame_w;
  const int64_t nu = nf * factor * factor;
  if ((int64_t)factor * frame_h * factor * frame_w >= ((int64_t)1 << 31))
    return fail(EM_EINVAL, "up-sampled frame of 2^31 pixels or more");
  int rc;
  if ((rc = check_device_range(y, (size_t)nf * sizeof(float), "y"))) return rc;
  if ((rc = check_device_range(v, (size_t)nf * sizeof(float), "v"))) return rc;
  if ((rc = check_device_range(y_up, (size_t)nu * sizeof(float), "y_up"))) return rc;
  if ((rc = check_device_range(v_up, (size_t)nu * sizeof(float), "v_up"))) return rc;
  EM_HIP(launch_upsample(y, v, n_frames, frame_h, frame_w, factor, y_up, v_up,
                         static_cast<hipStream_t>(stream)));
  return EM_OK;
}

void em_psf_defaults(em_psf_problem* p) {
  if (!p) return;
  p->n_frames = 1;
  p->psf_k = 43;
  p->out_k = 43;
  p->factor = 2;
  p->n_steps = 2000;
  p->sigma = 2.f;
  p->lambda = 1e-2f;
  p->lr = 1e-2f;
  p->lr_decay = 1e-2f;
  p->beta1 = 0.9f;
  p->beta2 = 0.999f;
  p->eps = 1e-7f;
}

int em_psf_fit(const em_psf_problem* p, const float* f, const float* h0, float* h,
               double* objective, void* stream) {
  if (!p) return fail(EM_EINVAL, "problem is NULL");
  const int kf = p->psf_k, kh = p->out_k;
  if (p->n_frames < 1 || p->n_frames > (1 << 20)) return fail(EM_EINVAL, "n_frames out of range");
  if (kf < 1 || kf > PSF_K_MAX || kf % 2 == 0 || kh < 1 || kh > PSF_K_MAX || kh % 2 == 0)
    return fail(EM_EINVAL, "psf_k and out_k must be odd and in 1..%d", PSF_K_MAX);
  if (p->factor < 1 || p->factor > 4) return fail(EM_EINVAL, "factor must be 1..4");
  if (p->n_steps < 0) return fail(EM_EINVAL, "n_steps < 0");
  if (!(p->sigma >= 0.f && p->sigma <= 8.f)) return fail(EM_EINVAL, "sigma must be in [0, 8]");
  if (!(p->lambda >= 0.f) || !std::isfinite(p->lambda)) return fail(EM_EINVAL, "lambda must be >= 0");
  if (!(p->lr >= 0.f) || !std::isfinite(p->lr)) return fail(EM_EINVAL, "lr must be >= 0");
  if (!(p->lr_decay > 0.f) || !std::isfinite(p->lr_decay)) return fail(EM_EINVAL, "lr_decay must be > 0");
  if (!(p->beta1 >= 0.f && p->beta1 < 1.f) || !(p->beta2 >= 0.f && p->beta2 < 1.f))
    return fail(EM_EINVAL, "beta1 and beta2 must be in [0, 1)");
  if (!(p->eps > 0.f) || !std::isfinite(p->eps)) return fail(EM_EINVAL, "eps must be > 0");
  const size_t fb = (size_t)p->n_frames * kf * kf * sizeof(float);
  const size_t hb = (size_t)p->n_frames * kh * kh * sizeof(float);
  int rc;
  if ((rc = check_device_range(f, fb, "f"))) return rc;
  if ((rc = check_device_range(h, hb, "h"))) return rc;
  if (h0 && (rc = check_device_range(h0, hb, "h0"))) return rc;
  if (objective && (rc = check_device_range(objective, (size_t)p->n_frames * sizeof(double), "objective")))
    return rc;
  PsfParams P;
  P.n = p->n_frames;
  P.kf = kf;
  P.kh = kh;
  P.D = p->factor;
  P.S = p->n_steps;
  P.sigma = p->sigma;
  P.lam = p->lambda;
  P.lr = p->lr;
  P.decay = p->lr_decay;
  P.b1 = p->beta1;
  P.b2 = p->beta2;
  P.eps = p->eps;
  EM_HIP(launch_psf_fit(P, f, h0, h, objective, static_cast<hipStream_t>(stream)));
  return EM_OK;
}

}  // extern "C"

// ---- allocation-free entry point ---------------------------------------------
// The scratch of em_run_noalloc: a file-scope device array that every GPU the
// library runs on holds until the process ends.  In host code `em_noalloc_scratch`
// names a host-side stand-in; its device address on the current device comes
// from hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) char em_noalloc_scratch[EM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;                        // serialises calls (one array per GPU)
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};  // device address per device, once known
}  // namespace

extern "C" int em_run_noalloc(const em_problem* p, const float* y, const float* v,
                              const float* psf, const float* x0, float* x, int32_t n_iter,
                              double* loglik_trace, void* stream) {
  if (n_iter < 0) return fail(EM_EINVAL, "n_iter < 0");
  Geometry g;
  const char* why = nullptr;
  if (!make_geometry(p, &g, &why)) return fail(EM_EINVAL, "invalid problem: %s", why);
  const size_t need = make_layout(g, make_plan(g)).total;
  if (need > EM_NOALLOC_SCRATCH_BYTES)
    return fail(EM_ENOMEM,
                "the problem needs %zu bytes of scratch; em_run_noalloc holds %zu (use em_init "
                "with a workspace of em_workspace_bytes())",
                need, (size_t)EM_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  EM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(EM_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(em_noalloc_scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(EM_EDEVICE, "scratch address on device %d: %s", dev, hipGetErrorString(e));
    g_noalloc_ptr[dev] = ptr;
  }
  em_ctx c{};
  c.no_graph = true;   // eager launches: nothing is instantiated
  int rc = setup_job(&c, p, y, v, psf, x0, x, g_noalloc_ptr[dev], EM_NOALLOC_SCRATCH_BYTES,
                     stream, false, false);
  if (rc != EM_OK) return rc;
  if ((rc = em_iterate(&c, n_iter, loglik_trace)) != EM_OK) return rc;
  // the next call reuses the array: this one's kernels must be done
  EM_HIP(hipStreamSynchronize(c.stream));
  return EM_OK;
}
