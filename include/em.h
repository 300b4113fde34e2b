/*
 * em.h -- C ABI of libem.so: the MI355X (gfx950) hot path of the multi-frame
 * expectation-maximisation deconvolution and super-resolution method of
 * Sukurdeep, Navarro & Budavari, arXiv:2302.05804, Sec. 2.
 *
 * What the library computes (paper notation):
 *   exposures y^(t), PSFs f^(t) (or super-resolved h^(t)), variance maps v^(t),
 *   t = 1..n; inverse-variance weights u^(t) = 1/v^(t) (text after Eq. (2)).
 *   Image model, Eq. (1):  y^(t) = f^(t) * x + noise, noise ~ N(0, v^(t)).
 *   Super-resolution model, Eq. (3):  y^(t) = D(h^(t) * x) + noise, with D a
 *   2x2 box sum from the latent grid (x) to the frame grid (y).
 *   One EM iteration, the multiplicative update of Eq. (2):
 *       x <- x (.) max(B, 0) / Dn,
 *       B  = sum_t F_t^T (u_t (.) y_t)          (constant, formed once),
 *       Dn = sum_t F_t^T (u_t (.) F_t x),
 *   where F_t x = D(f_t * x) (D = identity when sr = 1).  The weights act on
 *   the frame grid before the adjoint; this is the majorise-minimise step of the
 *   Gaussian likelihood of Eq. (1) (the paper's Eq. (2) typesets u outside
 *   F^T, which coincides when each v^(t) is constant; weight mode
 *   EM_W_LITERAL reproduces the typeset form, sr = 1 only).
 *   Guards: x_j = 0 stays 0 (zeros are absorbing); x_j > 0 with Dn_j = 0 (a
 *   pixel no unmasked frame pixel sees) keeps its value.
 *   Log-likelihood, from Eq. (1):
 *       l(x) = -1/2 sum_t sum_{u>0} [ u (y - F_t x)^2 + ln(2 pi v) ].
 *
 * Conventions:
 *   - Convolution is a true 2-D convolution with an odd K x K kernel whose
 *     centre is c = (K-1)/2, zero-filled outside the latent grid, output the
 *     size of the grid ("same").  PSFs live on the latent grid.
 *   - The latent grid is (sr*frame_h) x (sr*frame_w); frame pixel (I,J)
 *     covers latent pixels (sr*I + p, sr*J + q), p,q < sr.
 *   - All images are contiguous row-major float32.  Exposures and variances are
 *     n x frame_h x frame_w, PSFs n x K x K, latent images H_lat x W_lat.
 *   - v = +inf marks a masked pixel (u = 0); y there is never read as a
 *     number (it may be NaN).  Any other v must be finite and > 0, and an
 *     unmasked y must be finite; PSF taps must be finite and >= 0.
 *
 * Streams: a `stream` argument is a hipStream_t passed as void* (NULL is the
 * default stream).  Device pointers are plain HIP device addresses.
 *
 * Errors: every entry point returns EM_OK (0) or a negative EM_E* code and
 * never throws.  em_last_error() returns a thread-local text for the last
 * failure on the calling thread.  Device errors from asynchronous work surface
 * at the next synchronising call (em_init, em_iterate with a trace,
 * em_loglik, em_sync).
 *
 * Threading: an em_ctx must be used by one thread at a time.
 */
#ifndef EM_H
#define EM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define EM_OK         0
#define EM_EINVAL    (-1)   /* bad argument or invalid input data            */
#define EM_ENOMEM    (-2)   /* workspace / budget too small                   */
#define EM_EDEVICE   (-3)   /* HIP runtime error (text in em_last_error)      */
#define EM_EAGAIN    (-4)   /* serving: job not finished yet                  */
#define EM_ECANCELED (-5)   /* serving: job cancelled                         */
#define EM_ENOTSUP   (-6)   /* combination not provided by this build         */

/* arithmetic of the two convolutions (the update is always FP32, the
 * log-likelihood and convergence sums always FP64) */
#define EM_FP32        0    /* FP32 products, FP32 accumulation               */
#define EM_BF16_SPLIT  1    /* BF16 MFMA, image and PSF split into hi+lo,
                               three products (hi hi, hi lo, lo hi), FP32
                               accumulation.  K = 43, sr = 1, not served: when
                               every frame's PSF keeps at most 1/16 of its
                               mass outside the 21 kernel rows nearest the
                               centre (checked at set-up), the taps on the
                               other rows take the hi hi product alone       */
#define EM_FP16_SPLIT  2    /* FP16 MFMA: image operand in binary16 with a
                               power-of-two scale (per staged tile of x; for
                               the adjoint of a Gaussian iteration with sr = 1,
                               or sr = 2 and 8 or more frames, r written by the
                               forward in binary16 with a per-frame scale
                               fixed from a bound on u_t F_t x), PSF split into
                               binary16 hi+lo with a power-of-two scale per
                               frame, FP32 accumulation, scales removed exactly
                               in the epilogue.  Two products (hi, lo) on the
                               kernel rows near the centre (K = 43: the 21
                               rows within 10 of it; sr = 2: rows 11..32 of the
                               44-row stride-2 kernel), the hi part alone on
                               the others                                    */
#define EM_BF16        3    /* plain BF16 MFMA (ablation; below 1e-3 accuracy) */

/* placement of the inverse-variance weights, and the noise model */
#define EM_W_ADJOINT   0    /* sum_t F_t^T (u_t (.) .)  (default)              */
#define EM_W_LITERAL   1    /* sum_t u_t (.) F_t^T (.)  (Eq. (2) as typeset, sr=1):
                               B = sum_t u_t (.) F_t^T yhat_t and
                               Dn = sum_t u_t (.) F_t^T F_t x, u_t read on the
                               latent grid (= the frame grid for sr = 1).  Each
                               frame's adjoint goes to its own plane (the
                               workspace holds n latent planes) and the planes
                               are summed with their weights in frame order;
                               l(x) is that of Eq. (1).  Not served by
                               em_server (EM_ENOTSUP); EM_ENOTSUP for sr = 2. */
#define EM_W_STUDENT_T 2    /* Student-t noise with nu degrees of freedom and
                               scale v (the heavier-tailed noise the paper
                               names as future work): every iteration gives
                               each observed pixel the E-step weight
                               w = (nu+1)/(nu + u (y - F_t x)^2) of the
                               Gaussian scale-mixture form (Lange, Little &
                               Taylor, 1989) and runs the update of Eq. (2)
                               with u w in place of u, the numerator
                               B = sum_t F_t^T(u_t w_t y_t) formed again;
                               l(x) is the Student-t log-likelihood
                               sum_{u>0} [lgamma((nu+1)/2) - lgamma(nu/2)
                               - ln(nu pi v)/2 - (nu+1)/2 ln(1 + u (y-F_t x)^2/nu)].
                               An iteration costs one forward and two adjoint
                               passes; the workspace holds one more frame-sized
                               plane.  Served by em_server like the default. */

typedef struct em_ctx em_ctx;
typedef struct em_server em_server;
typedef int64_t em_job_id;

typedef struct {
    int32_t n_frames;     /* n >= 1                                          */
    int32_t frame_h;      /* exposure rows    >= 1                           */
    int32_t frame_w;      /* exposure columns >= 1                           */
    int32_t psf_k;        /* odd, 1 <= K <= 43                               */
    int32_t sr;           /* super-resolution factor: 1 or 2 (Eq. (3))       */
    int32_t precision;    /* EM_FP32, EM_BF16_SPLIT, EM_FP16_SPLIT, EM_BF16   */
    int32_t weight_mode;  /* EM_W_ADJOINT, EM_W_LITERAL (sr = 1), EM_W_STUDENT_T */
    float nu;             /* EM_W_STUDENT_T: degrees of freedom in (0, 1e30];
                             ignored otherwise                                 */
} em_problem;

/* Library build / device description (NUL-terminated, static storage). */
const char* em_version(void);

/* Thread-local text of the last error on this thread ("" if none). */
const char* em_last_error(void);

/*
 * Device bytes the library needs beyond the caller's buffers for problem p
 * (weights, weighted model images, numerator B, coefficient tables, FP64
 * partial sums).  Returns 0 for an invalid problem.
 */
size_t em_workspace_bytes(const em_problem* p);

/*
 * Set up one deconvolution job (Sec. 2: data y, f, v; initial guess x^(0)).
 *   y, v      device, n x frame_h x frame_w float32 (caller-owned, borrowed
 *             until em_destroy; not modified)
 *   psf       device, n x K x K float32 on the latent grid (borrowed)
 *   x0        device latent image, or NULL for the flat guess
 *             x0 = max(mu, 1e-3) / sr^2, mu = sum u y / sum u
 *             (x0 must be finite and >= 0; zeros stay zero)
 *   x         device latent image (the iterate; written here, updated in
 *             place by em_iterate; borrowed)
 *   workspace device buffer of ws_bytes >= em_workspace_bytes(p), 256-byte
 *             aligned (borrowed)
 *   stream    hipStream_t (as void*) on which all of the job's work runs
 * Computes u, B and x^(0) on the stream and synchronises it to validate the
 * data.  Returns EM_EINVAL for a bad problem, NULL pointers or invalid data,
 * EM_ENOMEM if ws_bytes is too small, EM_ENOTSUP for an unsupported
 * precision / weight mode combination, EM_EDEVICE on a HIP error.
 */
int em_init(em_ctx** out, const em_problem* p,
            const float* y, const float* v, const float* psf,
            const float* x0, float* x,
            void* workspace, size_t ws_bytes, void* stream);

/*
 * Run n_iter >= 0 iterations of the multiplicative update of Eq. (2)
 * asynchronously on the job's stream.  If loglik_trace (host, n_iter doubles)
 * is non-NULL, loglik_trace[k-1] = l(x^(k-1)) for k = 1..n_iter, and the
 * call synchronises the stream before returning.
 */
int em_iterate(em_ctx* ctx, int32_t n_iter, double* loglik_trace);

/*
 * Like em_iterate, but stops after the first iteration k whose relative change
 * ||x^(k) - x^(k-1)||_2 / ||x^(k-1)||_2 is below tol (FP64 sums on the GPU;
 * the paper leaves the convergence criterion open, Sec. 2).  Checks every
 * `check_every` iterations (>= 1).  Writes the iterations run to *iters_done and,
 * if relchange_trace (host, max_iter doubles) is non-NULL, the relative
 * change of every iteration run.  Synchronous.
 */
int em_iterate_tol(em_ctx* ctx, int32_t max_iter, double tol, int32_t check_every,
                   int32_t* iters_done, double* loglik_trace, double* relchange_trace);

/* l(x) at the current iterate, FP64 (synchronous). */
int em_loglik(em_ctx* ctx, double* out);

/*
 * Diagnostics of the two frame sums of Eq. (2) at the current iterate: writes
 * B (if B_out != NULL) and Dn (if Dn_out != NULL) as device float32 latent
 * images.  Asynchronous on the job's stream; does not change the iterate.
 */
int em_terms(em_ctx* ctx, float* B_out, float* Dn_out);

/*
 * Measurement: runs n_iter iterations like em_iterate (no trace) and times
 * every kernel launch of the iteration with HIP events recorded on the job's
 * stream.  Writes the mean duration in milliseconds per launch of
 *   phase_ms[0]  the forward kernel  (F_t x, weighting; all frames)
 *   phase_ms[1]  the adjoint kernel  (F_t^T r, frame sum; fused update if
 *                                     the adjoint is not split over frame groups)
 *   phase_ms[2]  the separate update kernel (0 when fused)
 *   phase_ms[3]  the whole iteration
 * Under EM_W_STUDENT_T phase_ms[0] is the forward kernel with the E-step
 * weights in its epilogue, and the numerator's adjoint counts in phase_ms[3]
 * only.
 * Synchronous.
 */
int em_profile(em_ctx* ctx, int32_t n_iter, double* phase_ms);

/*
 * Kernel variants of the matrix-core precisions (tile / wave layouts that
 * compute the same sums; results may differ from one variant to another at the
 * rounding level).  em_variant_count() gives their number; em_set_variants
 * selects one per direction (0 = forward, 1 = adjoint) for ctx.
 */
int em_variant_count(void);
int em_set_variants(em_ctx* ctx, int32_t fwd_variant, int32_t adj_variant);

/*
 * Autotuner: times every variant of the forward and the adjoint kernel on the
 * job's own data (n_rep launches each after one warm-up, HIP events on the
 * job's stream; the iterate x is not modified) and selects the fastest for
 * ctx alone.  Every job starts on variants 0 / 0, whatever other jobs of the
 * process chose, so its arithmetic never depends on them.  Writes the chosen
 * variants and, if ms != NULL, the mean launch times
 * ms[dir * em_variant_count() + v].  Synchronous.
 * EM_ENOTSUP for FP32 (one variant).
 */
int em_autotune(em_ctx* ctx, int32_t n_rep, int32_t* fwd_variant, int32_t* adj_variant,
                double* ms);

/*
 * Host-only self-check (no GPU needed): builds every launch descriptor the
 * library would use for problem p (iteration, autotuning, stand-alone operators,
 * serving plan; every kernel variant) and checks each against the grid it is
 * launched on and the workspace sizes.  EM_OK, or EM_EINVAL with the reason.
 */
int em_check_plan(const em_problem* p);

/* Wait for the job's stream; reports asynchronous device errors. */
int em_sync(em_ctx* ctx);

/* Release library state of the job (caller buffers are not freed). */
int em_destroy(em_ctx* ctx);

/*
 * For callers that cannot allocate memory (tight serving loops, harnesses
 * that forbid hipMalloc): one job in one call, em_init followed by
 * em_iterate(n_iter, loglik_trace), with the workspace taken from a scratch
 * array of EM_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends.  The call allocates nothing (no hipMalloc,
 * no graph instantiation: the iterations are launched one by one) and
 * creates no em_ctx; the caller passes y, v, psf, x0 (or NULL for the flat
 * start) and x exactly as for em_init.  Results are those of em_init +
 * em_iterate with the default kernel variants.
 * Limits: EM_ENOMEM when em_workspace_bytes(p) > EM_NOALLOC_SCRATCH_BYTES.
 * One array per GPU: calls are serialised inside the library and each one
 * synchronises `stream` before returning, so the next call may reuse the
 * array; work of the caller that overlaps a call on the same GPU must not
 * touch it (calls that overlapped on one GPU would race).  The array keeps
 * the last call's contents; everything a call reads is written by that call
 * first.  Synchronous; not capturable (it reads validation flags back).
 */
#define EM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int em_run_noalloc(const em_problem* p, const float* y, const float* v, const float* psf,
                   const float* x0, float* x, int32_t n_iter, double* loglik_trace,
                   void* stream);

/*
 * Stand-alone operators, for checking: F_t x and F_t^T r for every frame.
 *   psf: device n x K x K; x, s: device latent images n x H_lat x W_lat for
 *   em_adjoint_op output and one latent image for em_forward_op input;
 *   m, r: device n x frame_h x frame_w.  `workspace` must hold
 *   em_workspace_bytes(p) bytes.  Asynchronous on `stream`.
 */
int em_forward_op(const em_problem* p, const float* psf, const float* x, float* m,
                  void* workspace, size_t ws_bytes, void* stream);
int em_adjoint_op(const em_problem* p, const float* psf, const float* r, float* s,
                  void* workspace, size_t ws_bytes, void* stream);

/*
 * Up-sampled exposures for the super-resolution run the paper describes after
 * Eq. (4) (arXiv:2302.05804, Sec. 2): the super-resolved PSFs h and up-sampled
 * exposures y^D take the place of f and y in the update of Eq. (2), with no
 * down-sampling operator; the job is then an ordinary sr = 1 problem on the
 * fine grid (frame_h = factor * the exposures' rows, PSFs h).  The paper does
 * not say how y is up-sampled; each frame pixel is replicated into a
 * factor x factor block of fine pixels that share its flux:
 *     y_up[t][f i + p][f j + q] = y[t][i][j] / f^2,
 *     v_up[t][f i + p][f j + q] = v[t][i][j] / f^4   (variance of y / f^2),
 * binary32 quotients, so masked pixels (v = +inf) stay masked.
 *   y, v: device n x frame_h x frame_w (caller-owned, read only);
 *   y_up, v_up: device n x (factor frame_h) x (factor frame_w), written.
 * factor: 2, 3 or 4.  EM_EINVAL for NULL pointers, buffers that do not fit in
 * their device allocation, non-positive sizes or another factor (a buffer
 * carved out of a larger allocation is checked against that allocation).  Asynchronous on `stream` (hipStream_t as void*,
 * NULL = default stream); allocates nothing.
 */
int em_upsample(int32_t n_frames, int32_t frame_h, int32_t frame_w, int32_t factor,
                const float* y, const float* v, float* y_up, float* v_up, void* stream);

/*
 * Super-resolved PSFs, Eq. (4) (arXiv:2302.05804, Sec. 2): for every frame t,
 *     h_t = argmin_{h >= 0} sum_IJ ([D(h * g)]_IJ - f_t[I][J])^2 + lambda |grad h|^2,
 * fitted by projected Adam (Kingma & Ba, 2015, Algorithm 1), the solver the
 * paper uses.  Readings of what the paper leaves open:
 *   - f_t is psf_k x psf_k on the frame grid, h_t out_k x out_k on the fine
 *     grid (both odd).  The data term covers the factor*psf_k fine stamp that
 *     D (factor x factor block sums, coarse pixel I = fine rows factor*I ..
 *     factor*I + factor - 1) maps onto f's stamp; h's centre sits on fine
 *     pixel factor*(psf_k-1)/2, the phase of D in Eq. (3).  h*g is a true
 *     convolution; what falls outside the fine stamp is not seen.
 *   - g: isotropic Gaussian, standard deviation `sigma` fine pixels (the
 *     paper's width; sigma = factor by default), sampled at pixel centres
 *     within ceil(4 sigma), unit sum; sigma = 0 is the unit impulse.
 *   - |grad h|^2: squared forward differences of h extended by zeros, over
 *     every pair of 4-neighbours with a pixel on the stamp.
 *   - Each Adam step is followed by h = max(h, 0).  Step k of n_steps uses
 *     lr * max(f_t) * lr_decay^((k-1)/(n_steps-1)).
 *   - Start: f replicated into factor x factor blocks of value f/factor^2
 *     (negative values set to 0), cropped to out_k x out_k about the anchor;
 *     or h0 when given.
 * Arguments (device pointers, row-major binary32):
 *   f: n_frames x psf_k x psf_k, finite (read only);
 *   h0: n_frames x out_k x out_k start, or NULL for the start above;
 *   h: n_frames x out_k x out_k result (written);
 *   objective: n_frames doubles, the objective at the result, or NULL.
 * One workgroup per frame; asynchronous on `stream` (hipStream_t as void*,
 * NULL = default stream); allocates nothing.  EM_EINVAL for NULL f or h,
 * buffers that do not fit their device allocation, even or out-of-range
 * sizes (psf_k, out_k in 1..63; factor 1..4; the EM kernels take PSFs up to
 * 43), sigma outside [0, 8], lambda < 0, lr < 0, lr_decay <= 0, beta outside
 * [0, 1), eps <= 0 or n_steps < 0.
 */
typedef struct {
  int32_t n_frames; /* PSFs to fit */
  int32_t psf_k;    /* side of f_t (odd) */
  int32_t out_k;    /* side of h_t (odd) */
  int32_t factor;   /* Delta of Eq. (3) */
  int32_t n_steps;  /* Adam steps */
  float sigma;      /* std of g in fine pixels */
  float lambda;     /* weight of the gradient penalty */
  float lr;         /* first step, relative to max f_t */
  float lr_decay;   /* last step / first step */
  float beta1, beta2, eps; /* Adam */
} em_psf_problem;

/* Fill p with the defaults: factor 2, sigma 2, lambda 1e-2, 2000 steps,
 * lr 1e-2, lr_decay 1e-2, beta1 0.9, beta2 0.999, eps 1e-7, out_k 43,
 * psf_k 43, n_frames 1. */
void em_psf_defaults(em_psf_problem* p);

int em_psf_fit(const em_psf_problem* p, const float* f, const float* h0, float* h,
               double* objective, void* stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of deconvolution jobs on one GPU.
 *
 * A server owns one device arena of hbm_budget bytes (allocated once) and a
 * worker thread.  Jobs are admitted in arrival order whenever one of
 * max_slots slots and enough of the arena are free; admitted jobs keep their
 * inputs, iterate and workspace resident and advance together, one EM
 * iteration (Eq. (2)) per round, in one batched launch per kernel family
 * (captured in a HIP graph while the set of jobs is unchanged).  A finished
 * job's iterate and final log-likelihood are copied to host memory and its
 * arena space is reused at once.  Each job's result does not depend on what
 * else runs (fixed per-shape launch plan, no cross-job reductions).
 * All em_server calls are thread-safe.
 * ------------------------------------------------------------------------ */

/* stream: hipStream_t (as void*) for the server's work, or NULL for a stream
 * the server creates.  EM_ENOMEM if the budget cannot be allocated. */
int em_server_create(em_server** out, size_t hbm_budget, int32_t max_slots, void* stream);

/* Stops the worker (pending and running jobs are cancelled) and frees all. */
int em_server_destroy(em_server* server);

/* Device bytes a job of problem p takes from the server's budget. */
size_t em_job_bytes(const em_problem* p);

/*
 * Queue one job (non-blocking).  y_host, v_host (n x frame_h x frame_w) and
 * psf_host (n x K x K) are host float32 arrays copied before the call returns
 * (the caller may free them).  The starting guess is the flat rule of
 * em_init.  Returns EM_ENOMEM if the job can never fit the budget, EM_EINVAL /
 * EM_ENOTSUP for a bad problem (data errors are reported by em_poll/em_wait).
 */
int em_submit(em_server* server, const em_problem* p, const float* y_host, const float* v_host,
              const float* psf_host, int32_t n_iter, em_job_id* out);

/*
 * EM_OK when the job is done: copies its iterate (H_lat x W_lat float32) to
 * x_host_out and its final log-likelihood l(x^(n_iter)) to loglik_out (either
 * may be NULL); EM_EAGAIN while queued or running; EM_ECANCELED; or the
 * job's error.  em_wait blocks until the job leaves the pending states.
 */
int em_poll(em_server* server, em_job_id id, float* x_host_out, double* loglik_out);
int em_wait(em_server* server, em_job_id id, float* x_host_out, double* loglik_out);

/* Cancel a queued or running job (running jobs stop at the next round). */
int em_cancel(em_server* server, em_job_id id);

/* Forget a finished job and free its host result (EM_EAGAIN while it is
 * pending or another thread is still inside em_wait for it). */
int em_release(em_server* server, em_job_id id);

/* Steady-clock seconds at which the job was submitted, admitted, finished. */
int em_job_times(em_server* server, em_job_id id, double* t_submit, double* t_admit,
                 double* t_done);

/* stats[8]: queued, active, done, failed, cancelled, rounds run, round graphs
 * built, arena bytes in use. */
int em_server_stats(em_server* server, int64_t* stats);

/* Seconds the server's worker has spent, since creation, in each phase:
 * sec[0] admission (input upload, set-up of u, B and x0), sec[1] rebuilding
 * the round after the set of jobs changed (descriptors, graph capture),
 * sec[2] rounds (launch to completion of the batched iterations), sec[3]
 * finishing jobs (final log-likelihood, result copy to the host). */
int em_server_phase_seconds(em_server* server, double* sec);

/* Host staging of submitted inputs.  The server holds a pinned host area of
 * a quarter of hbm_budget (at most 2 GiB; none if pinned memory cannot be
 * allocated); em_submit copies a job's y and v there when it has room, so
 * that their upload at admission is an asynchronous DMA, else into pageable
 * memory.  A job's range is freed once its upload has completed.  out[3]:
 * staging bytes, jobs staged there, jobs staged in pageable memory. */
int em_server_staging(em_server* server, int64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* EM_H */
