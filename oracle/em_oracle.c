/*
 * em_oracle.c -- TEST INFRASTRUCTURE, not part of the product path.
 *
 * A plain, slow, single-threaded FP64 CPU reference of the multi-frame EM
 * deconvolution / super-resolution iteration of Sukurdeep, Navarro & Budavari,
 * "A Flexible Expectation Maximization Framework for Fast, Scalable and
 * High-fidelity Multi-frame Astronomical Image Deconvolution" (arXiv:2302.05804),
 * Sec. 2, Eqs. (1)-(3).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Every operator is written as its textbook definition (a sum over taps, with
 * loop bounds clipped to the image), evaluated pixel by pixel, in double.
 * Inputs that arrive as FP32 data (exposures, variances, PSFs, an initial
 * guess) are read as float and widened exactly to double.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - F_t x = D(f_t * x): true 2-D convolution, odd K, centre c=(K-1)/2,
 *    zero-filled outside the latent grid, output the size of the latent grid
 *    ("same"); D = identity for sr=1, a 2x2 box SUM for sr=2 where frame pixel
 *    I covers latent rows 2I and 2I+1 (Eq. (3)).
 *  - u = 1/v; v = +inf marks a masked pixel, u = 0 there, and y is replaced by
 *    0 there (it may hold NaN).
 *  - The weights act on the frame grid before the adjoint (the
 *    majorise-minimise step of the Gaussian likelihood of Eq. (1)):
 *        x <- x * max(B, 0) / Dn,  B = sum_t F_t^T (u_t y_t),
 *                                  Dn = sum_t F_t^T (u_t F_t x).
 *    The as-typeset form of Eq. (2), u_t (F_t^T y_t) / u_t (F_t^T F_t x) with
 *    u applied on the latent grid, is kept as weight mode 1 (sr=1 only).
 *  - Guards: x_j = 0 stays 0; x_j > 0 with Dn_j = 0 keeps x_j; otherwise
 *    q_j = max(B_j,0)/Dn_j is formed first and then x_j*q_j.
 *  - Log-likelihood of Eq. (1):
 *        l(x) = -1/2 sum_t sum_{u>0} [ u (y - F_t x)^2 + ln(2 pi v) ].
 *  - Flat initial guess: mu = sum u y / sum u over all frames and pixels,
 *    x0 = max(mu, 1e-3) / sr^2.
 *  - Frames are summed in the order t = 0 .. n-1.
 *  - The super-resolution run the paper describes after Eq. (4) (exposures
 *    up-sampled to the fine grid, no D): em_oracle_upsample below.
 *  - The super-resolved PSFs of Eq. (4), fitted by projected Adam:
 *    em_oracle_psf_* at the end of this file, with their own readings.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EMO_PI 3.14159265358979323846

static int imax(int a, int b) { return a > b ? a : b; }
static int imin(int a, int b) { return a < b ? a : b; }

/* floor division for possibly negative numerators, positive d */
static int fdiv(int a, int d) { return (a >= 0) ? a / d : -((-a + d - 1) / d); }

/* ---------------------------------------------------------------------------
 * Weights (text following Eq. (2): u = 1/v).  Returns the number of invalid
 * pixels: an unmasked v that is <= 0, NaN or -inf, or an unmasked y that is
 * not finite.
 * ------------------------------------------------------------------------- */
long em_oracle_weights(long npix, const float* y, const float* v, double* u, double* yhat)
{
    long bad = 0;
    for (long p = 0; p < npix; ++p) {
        double vv = (double)v[p];
        if (isinf(vv) && vv > 0) {           /* masked */
            u[p] = 0.0;
            yhat[p] = 0.0;
            continue;
        }
        if (!(vv > 0.0) || !isfinite(vv) || !isfinite((double)y[p])) {
            ++bad;
            u[p] = 0.0;
            yhat[p] = 0.0;
            continue;
        }
        u[p] = 1.0 / vv;
        yhat[p] = (double)y[p];
    }
    return bad;
}

/* ---------------------------------------------------------------------------
 * Forward operator at one frame pixel (Eq. (1) for sr=1, Eq. (3) for sr=2):
 *   (F x)[I,J] = sum_{p,q<sr} sum_{a,b} f[a,b] x[sr I + p + c - a, sr J + q + c - b]
 * with x = 0 outside the Hl x Wl latent grid.
 * ------------------------------------------------------------------------- */
double em_oracle_forward_at(int K, int sr, int Hl, int Wl, const double* f, const double* x,
                            int I, int J)
{
    const int c = (K - 1) / 2;
    double acc = 0.0;
    for (int p = 0; p < sr; ++p) {
        for (int q = 0; q < sr; ++q) {
            const int i = sr * I + p, j = sr * J + q;
            /* need 0 <= i + c - a < Hl  and  0 <= a < K */
            const int a_lo = imax(0, i + c - Hl + 1), a_hi = imin(K - 1, i + c);
            const int b_lo = imax(0, j + c - Wl + 1), b_hi = imin(K - 1, j + c);
            for (int a = a_lo; a <= a_hi; ++a)
                for (int b = b_lo; b <= b_hi; ++b)
                    acc += f[a * K + b] * x[(long)(i + c - a) * Wl + (j + c - b)];
        }
    }
    return acc;
}

/* ---------------------------------------------------------------------------
 * Adjoint at one latent pixel:  (F^T r)[k,l] = (H^T D^T r)[k,l]
 *   (D^T r)[i,j] = r[floor(i/sr), floor(j/sr)]     (replicate)
 *   (H^T s)[k,l] = sum_{a,b} f[a,b] s[k - c + a, l - c + b]   (correlation)
 * with s = 0 outside the latent grid.
 * ------------------------------------------------------------------------- */
double em_oracle_adjoint_at(int K, int sr, int Hl, int Wl, const double* f, const double* r,
                            int k, int l)
{
    const int c = (K - 1) / 2;
    const int Wf = Wl / sr;
    double acc = 0.0;
    const int a_lo = imax(0, c - k), a_hi = imin(K - 1, Hl - 1 - k + c);
    const int b_lo = imax(0, c - l), b_hi = imin(K - 1, Wl - 1 - l + c);
    for (int a = a_lo; a <= a_hi; ++a) {
        const int i = k - c + a;
        for (int b = b_lo; b <= b_hi; ++b) {
            const int j = l - c + b;
            acc += f[a * K + b] * r[(long)fdiv(i, sr) * Wf + fdiv(j, sr)];
        }
    }
    return acc;
}

void em_oracle_forward(int K, int sr, int Hl, int Wl, const double* f, const double* x, double* m)
{
    const int Hf = Hl / sr, Wf = Wl / sr;
    for (int I = 0; I < Hf; ++I)
        for (int J = 0; J < Wf; ++J)
            m[(long)I * Wf + J] = em_oracle_forward_at(K, sr, Hl, Wl, f, x, I, J);
}

void em_oracle_adjoint(int K, int sr, int Hl, int Wl, const double* f, const double* r, double* s)
{
    for (int k = 0; k < Hl; ++k)
        for (int l = 0; l < Wl; ++l)
            s[(long)k * Wl + l] = em_oracle_adjoint_at(K, sr, Hl, Wl, f, r, k, l);
}

/* ---------------------------------------------------------------------------
 * Whole-problem helpers.  Shapes: y, v: n x Hf x Wf; f: n x K x K (float);
 * latent grid Hl = sr*Hf, Wl = sr*Wf.
 * ------------------------------------------------------------------------- */
typedef struct {
    int n, Hf, Wf, K, sr;
    long nf, nl;           /* pixels per frame, latent pixels */
    double* u;             /* n * nf */
    double* yh;            /* n * nf */
    double* f;             /* n * K * K */
    double* m;             /* nf scratch */
    double* r;             /* nf scratch */
    double* s;             /* nl scratch */
    double lconst;         /* sum_{u>0} ln(2 pi v) */
    long bad;
} emo_state;

static void emo_free(emo_state* st)
{
    free(st->u); free(st->yh); free(st->f); free(st->m); free(st->r); free(st->s);
}

static int emo_setup(emo_state* st, int n, int Hf, int Wf, int K, int sr,
                     const float* y, const float* v, const float* psf)
{
    memset(st, 0, sizeof(*st));
    st->n = n; st->Hf = Hf; st->Wf = Wf; st->K = K; st->sr = sr;
    st->nf = (long)Hf * Wf;
    st->nl = st->nf * sr * sr;
    st->u = (double*)malloc(sizeof(double) * n * st->nf);
    st->yh = (double*)malloc(sizeof(double) * n * st->nf);
    st->f = (double*)malloc(sizeof(double) * n * K * K);
    st->m = (double*)malloc(sizeof(double) * st->nf);
    st->r = (double*)malloc(sizeof(double) * st->nf);
    st->s = (double*)malloc(sizeof(double) * st->nl);
    if (!st->u || !st->yh || !st->f || !st->m || !st->r || !st->s) { emo_free(st); return -2; }
    st->bad = em_oracle_weights((long)n * st->nf, y, v, st->u, st->yh);
    for (long p = 0; p < (long)n * K * K; ++p) st->f[p] = (double)psf[p];
    double lc = 0.0;
    for (long p = 0; p < (long)n * st->nf; ++p)
        if (st->u[p] > 0.0) lc += log(2.0 * EMO_PI * (double)v[p]);
    st->lconst = lc;
    return 0;
}

/* l(x) of Eq. (1), summed over unmasked pixels, frames in order. */
static double emo_loglik(emo_state* st, const double* x)
{
    const int Hl = st->Hf * st->sr, Wl = st->Wf * st->sr;
    double quad = 0.0;
    for (int t = 0; t < st->n; ++t) {
        const double* ft = st->f + (long)t * st->K * st->K;
        em_oracle_forward(st->K, st->sr, Hl, Wl, ft, x, st->m);
        const double* ut = st->u + (long)t * st->nf;
        const double* yt = st->yh + (long)t * st->nf;
        for (long p = 0; p < st->nf; ++p)
            if (ut[p] > 0.0) {
                const double d = yt[p] - st->m[p];
                quad += ut[p] * d * d;
            }
    }
    return -0.5 * (quad + st->lconst);
}

/* Numerator of Eq. (2).  mode 0: B = sum_t F_t^T (u_t y_t);
 * mode 1 (sr=1): B = sum_t u_t (F_t^T y_t). */
static void emo_numerator(emo_state* st, int mode, double* B)
{
    const int Hl = st->Hf * st->sr, Wl = st->Wf * st->sr;
    for (long j = 0; j < st->nl; ++j) B[j] = 0.0;
    for (int t = 0; t < st->n; ++t) {
        const double* ft = st->f + (long)t * st->K * st->K;
        const double* ut = st->u + (long)t * st->nf;
        const double* yt = st->yh + (long)t * st->nf;
        if (mode == 0) {
            for (long p = 0; p < st->nf; ++p) st->r[p] = ut[p] * yt[p];
            em_oracle_adjoint(st->K, st->sr, Hl, Wl, ft, st->r, st->s);
            for (long j = 0; j < st->nl; ++j) B[j] += st->s[j];
        } else {
            em_oracle_adjoint(st->K, st->sr, Hl, Wl, ft, yt, st->s);
            for (long j = 0; j < st->nl; ++j) B[j] += ut[j] * st->s[j];
        }
    }
}

/* Denominator of Eq. (2) at x, plus (optionally) l(x) from the same F_t x. */
static void emo_denominator(emo_state* st, int mode, const double* x, double* Dn, double* loglik)
{
    const int Hl = st->Hf * st->sr, Wl = st->Wf * st->sr;
    double quad = 0.0;
    for (long j = 0; j < st->nl; ++j) Dn[j] = 0.0;
    for (int t = 0; t < st->n; ++t) {
        const double* ft = st->f + (long)t * st->K * st->K;
        const double* ut = st->u + (long)t * st->nf;
        const double* yt = st->yh + (long)t * st->nf;
        em_oracle_forward(st->K, st->sr, Hl, Wl, ft, x, st->m);
        for (long p = 0; p < st->nf; ++p)
            if (ut[p] > 0.0) {
                const double d = yt[p] - st->m[p];
                quad += ut[p] * d * d;
            }
        if (mode == 0) {
            for (long p = 0; p < st->nf; ++p) st->r[p] = ut[p] * st->m[p];
            em_oracle_adjoint(st->K, st->sr, Hl, Wl, ft, st->r, st->s);
            for (long j = 0; j < st->nl; ++j) Dn[j] += st->s[j];
        } else {
            em_oracle_adjoint(st->K, st->sr, Hl, Wl, ft, st->m, st->s);
            for (long j = 0; j < st->nl; ++j) Dn[j] += ut[j] * st->s[j];
        }
    }
    if (loglik) *loglik = -0.5 * (quad + st->lconst);
}

/* Multiplicative update of Eq. (2) with the non-negativity clamp and guards. */
static void emo_update(long nl, const double* B, const double* Dn, double* x,
                       double* dsq, double* xsq)
{
    double a = 0.0, b = 0.0;
    for (long j = 0; j < nl; ++j) {
        const double xo = x[j];
        double xn;
        if (xo == 0.0) {
            xn = 0.0;
        } else if (Dn[j] == 0.0) {
            xn = xo;
        } else {
            const double q = (B[j] > 0.0 ? B[j] : 0.0) / Dn[j];
            xn = xo * q;
        }
        a += (xn - xo) * (xn - xo);
        b += xo * xo;
        x[j] = xn;
    }
    if (dsq) *dsq = a;
    if (xsq) *xsq = b;
}

/* ---------------------------------------------------------------------------
 * Public entry points (called through ctypes from the test-suite).
 * ------------------------------------------------------------------------- */

/* ---------------------------------------------------------------------------
 * Up-sampled exposures of the super-resolution run the paper describes after
 * Eq. (4): the super-resolved PSFs h and up-sampled exposures y^D are used in
 * the update of Eq. (2) in place of f and y (no operator D).  The paper does
 * not say how y is up-sampled; the reading taken here replicates each frame
 * pixel into a D x D block of fine pixels that share its flux:
 *     y^D[t][D i + p][D j + q] = y[t][i][j] / D^2,
 *     v^D[t][D i + p][D j + q] = v[t][i][j] / D^4     (the variance of y / D^2),
 * with both quotients formed in binary32 (y and v are binary32 data).  A
 * masked pixel (v = +inf) stays masked.  Returns -1 for D outside [2, 4].
 * ------------------------------------------------------------------------- */
int em_oracle_upsample(int n, int Hf, int Wf, int D, const float* y, const float* v, float* yD,
                       float* vD)
{
    if (D < 2 || D > 4) return -1;
    const int Hu = D * Hf, Wu = D * Wf;
    const float d2 = (float)(D * D), d4 = (float)(D * D * D * D);
    for (int t = 0; t < n; ++t)
        for (int I = 0; I < Hu; ++I)
            for (int J = 0; J < Wu; ++J) {
                const long src = ((long)t * Hf + I / D) * Wf + J / D;
                const long dst = ((long)t * Hu + I) * Wu + J;
                yD[dst] = y[src] / d2;
                vD[dst] = v[src] / d4;
            }
    return 0;
}

/* Flat initial guess (see header comment).  Returns -1 on invalid input. */
double em_oracle_flat_x0(int n, int Hf, int Wf, int sr, const float* y, const float* v)
{
    const long np = (long)n * Hf * Wf;
    double num = 0.0, den = 0.0;
    for (long p = 0; p < np; ++p) {
        const double vv = (double)v[p];
        if (isinf(vv) && vv > 0) continue;
        if (!(vv > 0.0) || !isfinite(vv) || !isfinite((double)y[p])) return -1.0;
        num += (double)y[p] / vv;
        den += 1.0 / vv;
    }
    double mu = den > 0.0 ? num / den : 0.0;
    if (!(mu > 1e-3)) mu = 1e-3;
    return mu / (double)(sr * sr);
}

/* B of Eq. (2) (numerator), latent grid. */
int em_oracle_numerator(int n, int Hf, int Wf, int K, int sr, int mode,
                        const float* y, const float* v, const float* psf, double* B)
{
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    emo_numerator(&st, mode, B);
    emo_free(&st);
    return 0;
}

/* Dn of Eq. (2) (denominator) at x, latent grid. */
int em_oracle_denominator(int n, int Hf, int Wf, int K, int sr, int mode,
                          const float* y, const float* v, const float* psf,
                          const double* x, double* Dn)
{
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    emo_denominator(&st, mode, x, Dn, NULL);
    emo_free(&st);
    return 0;
}

/* l(x) of Eq. (1). */
int em_oracle_loglik(int n, int Hf, int Wf, int K, int sr,
                     const float* y, const float* v, const float* psf,
                     const double* x, double* out)
{
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    *out = emo_loglik(&st, x);
    emo_free(&st);
    return 0;
}

/*
 * Run k_max EM iterations of Eq. (2) from x (in: x^(0), out: x^(k_max)).
 * trace[k-1]     = l(x^(k-1))                 for k = 1..k_max (may be NULL)
 * relchange[k-1] = ||x^(k) - x^(k-1)|| / ||x^(k-1)||         (may be NULL)
 * Returns 0, -1 for invalid inputs, -2 for allocation failure.
 */
int em_oracle_run(int n, int Hf, int Wf, int K, int sr, int mode,
                  const float* y, const float* v, const float* psf,
                  double* x, int k_max, double* trace, double* relchange)
{
    if (n < 1 || Hf < 1 || Wf < 1 || K < 1 || (K % 2) == 0 || (sr != 1 && sr != 2)) return -1;
    if (mode == 1 && sr != 1) return -1;
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    double* B = (double*)malloc(sizeof(double) * st.nl);
    double* Dn = (double*)malloc(sizeof(double) * st.nl);
    if (!B || !Dn) { free(B); free(Dn); emo_free(&st); return -2; }
    emo_numerator(&st, mode, B);
    for (int k = 1; k <= k_max; ++k) {
        double ll = 0.0, a = 0.0, b = 0.0;
        emo_denominator(&st, mode, x, Dn, &ll);
        if (trace) trace[k - 1] = ll;
        emo_update(st.nl, B, Dn, x, &a, &b);
        if (relchange) relchange[k - 1] = b > 0.0 ? sqrt(a) / sqrt(b) : 0.0;
    }
    free(B); free(Dn);
    emo_free(&st);
    return 0;
}

/*
 * One iteration evaluated only at selected latent pixels (for checks at sizes
 * where a whole run is out of reach); Gaussian noise, or Student-t noise with
 * nu degrees of freedom (_t).  x0 (float, latent grid) is x^(0); for each
 * point (rows[i], cols[i]) writes B, Dn and x^(1) there (adjoint weighting).
 * Each F_t x value needed is evaluated on demand from its definition.
 */
static int emo_step_at(int n, int Hf, int Wf, int K, int sr, double nu,
                       const float* y, const float* v, const float* psf, const float* x0,
                       int npts, const int* rows, const int* cols,
                       double* B_out, double* Dn_out, double* x1_out)
{
    const int Hl = Hf * sr, Wl = Wf * sr, c = (K - 1) / 2;
    const long nl = (long)Hl * Wl;
    double* xd = (double*)malloc(sizeof(double) * nl);
    double* fd = (double*)malloc(sizeof(double) * K * K);
    if (!xd || !fd) { free(xd); free(fd); return -2; }
    for (long j = 0; j < nl; ++j) xd[j] = (double)x0[j];
    for (int pt = 0; pt < npts; ++pt) {
        const int k = rows[pt], l = cols[pt];
        double Bv = 0.0, Dv = 0.0;
        for (int t = 0; t < n; ++t) {
            for (int e = 0; e < K * K; ++e) fd[e] = (double)psf[(long)t * K * K + e];
            const float* yt = y + (long)t * Hf * Wf;
            const float* vt = v + (long)t * Hf * Wf;
            /* adjoint at (k,l): sum_{a,b} f[a,b] w[floor((k-c+a)/sr), floor((l-c+b)/sr)] */
            double bt = 0.0, dt = 0.0;
            for (int a = 0; a < K; ++a) {
                const int i = k - c + a;
                if (i < 0 || i >= Hl) continue;
                for (int b = 0; b < K; ++b) {
                    const int jj = l - c + b;
                    if (jj < 0 || jj >= Wl) continue;
                    const int I = i / sr, J = jj / sr;
                    const double vv = (double)vt[(long)I * Wf + J];
                    if (isinf(vv) && vv > 0) continue;            /* u = 0 */
                    if (!(vv > 0.0) || !isfinite((double)yt[(long)I * Wf + J])) {
                        free(xd); free(fd); return -1;
                    }
                    const double u = 1.0 / vv;
                    const double yv = (double)yt[(long)I * Wf + J];
                    const double mval = em_oracle_forward_at(K, sr, Hl, Wl, fd, xd, I, J);
                    /* Gaussian noise (nu <= 0): weight 1; Student-t: the E-step weight */
                    const double w = nu > 0.0 ? (nu + 1.0) / (nu + u * (yv - mval) * (yv - mval)) : 1.0;
                    bt += fd[a * K + b] * (u * w * yv);
                    dt += fd[a * K + b] * (u * w * mval);
                }
            }
            Bv += bt;
            Dv += dt;
        }
        const double xo = xd[(long)k * Wl + l];
        double xn;
        if (xo == 0.0) xn = 0.0;
        else if (Dv == 0.0) xn = xo;
        else xn = xo * ((Bv > 0.0 ? Bv : 0.0) / Dv);
        B_out[pt] = Bv; Dn_out[pt] = Dv; x1_out[pt] = xn;
    }
    free(xd); free(fd);
    return 0;
}

int em_oracle_step_at(int n, int Hf, int Wf, int K, int sr,
                      const float* y, const float* v, const float* psf, const float* x0,
                      int npts, const int* rows, const int* cols,
                      double* B_out, double* Dn_out, double* x1_out)
{
    return emo_step_at(n, Hf, Wf, K, sr, 0.0, y, v, psf, x0, npts, rows, cols, B_out, Dn_out, x1_out);
}

int em_oracle_step_at_t(int n, int Hf, int Wf, int K, int sr, double nu,
                        const float* y, const float* v, const float* psf, const float* x0,
                        int npts, const int* rows, const int* cols,
                        double* B_out, double* Dn_out, double* x1_out)
{
    if (!(nu > 0.0)) return -1;
    return emo_step_at(n, Hf, Wf, K, sr, nu, y, v, psf, x0, npts, rows, cols, B_out, Dn_out, x1_out);
}

/* ===========================================================================
 * Super-resolved PSFs, Eq. (4): for each frame t,
 *     h_t = argmin_{h >= 0}  sum_{I,J} ([D(h * g)]_{IJ} - f_t[I][J])^2
 *                            + lambda * sum (grad h)^2,
 * solved with Adam (Kingma & Ba, 2015, Algorithm 1), the solver the paper
 * names.  Readings of the points the paper leaves open:
 *  - Grids.  f is Kf x Kf on the frame grid (odd Kf, centre cf); h is Kh x Kh
 *    on the fine grid (odd Kh, centre ch).  The data term runs over the D*Kf x
 *    D*Kf fine stamp that D sums, block by block, onto f's stamp (coarse pixel
 *    I covers fine rows D*I .. D*I+D-1, as the operator D of Eq. (3)).  h is
 *    placed with its centre on fine pixel (D*cf, D*cf): a point source at
 *    fine pixel (D*I, D*J) seen through h and D lands on coarse pixel (I, J),
 *    the phase of D in Eq. (3).  h * g is a true convolution; the part of it
 *    outside the fine stamp is not seen by the data term.
 *  - g is an isotropic Gaussian whose standard deviation is sigma fine pixels
 *    (the paper's width Delta; sigma = D by default), sampled at pixel
 *    centres on a (2r+1)^2 stamp with r = ceil(4 sigma), and normalised to
 *    unit sum.  sigma = 0 makes g the unit impulse.
 *  - grad h: forward differences of h extended by zeros beyond its stamp, so
 *    the penalty is lambda times the sum of (h[i+1][j]-h[i][j])^2 and
 *    (h[i][j+1]-h[i][j])^2 over every pair of 4-neighbours with at least one
 *    pixel on the stamp.
 *  - h >= 0: each Adam step is followed by the projection max(h, 0).
 *  - Step size: lr_k = lr * max(f_t) * decay^((k-1)/(S-1)) at step k of S
 *    (an exponential schedule; a constant step leaves Adam circling the
 *    minimiser at its own scale).  max(f_t) makes lr relative to the PSF's
 *    scale.  beta1, beta2, eps as passed (0.9, 0.999, 1e-7 by default).
 *  - Start: f replicated into D x D blocks of fine pixels sharing its value
 *    (f/D^2, negative values set to 0), cropped to Kh x Kh about the anchor
 *    (zero where the crop leaves the stamp), unless h0 is given.
 * Everything below is evaluated from these definitions pixel by pixel.
 * ========================================================================= */

/* g of the header above; returns its side Kg (<= 2*33+1) and fills g[Kg*Kg]. */
int em_oracle_psf_gauss(double sigma, double* g)
{
    if (!(sigma >= 0.0) || sigma > 8.0) return -1;
    if (sigma == 0.0) { g[0] = 1.0; return 1; }
    const int r = (int)ceil(4.0 * sigma), Kg = 2 * r + 1;
    double s = 0.0;
    for (int i = 0; i < Kg; ++i)
        for (int j = 0; j < Kg; ++j) {
            const double di = i - r, dj = j - r;
            g[i * Kg + j] = exp(-(di * di + dj * dj) / (2.0 * sigma * sigma));
            s += g[i * Kg + j];
        }
    for (int i = 0; i < Kg * Kg; ++i) g[i] /= s;
    return Kg;
}

typedef struct {
    int Kf, Kh, D, Kg, S, anchor;
    double g[67 * 67];
} psf_geom;

static int psf_geom_init(psf_geom* G, int Kf, int Kh, int D, double sigma)
{
    if (Kf < 1 || Kh < 1 || Kf % 2 == 0 || Kh % 2 == 0 || D < 1 || D > 4) return -1;
    G->Kf = Kf; G->Kh = Kh; G->D = D;
    G->Kg = em_oracle_psf_gauss(sigma, G->g);
    if (G->Kg < 0) return -1;
    G->S = D * Kf;
    G->anchor = D * ((Kf - 1) / 2);
    return 0;
}

/* value of h at fine stamp pixel (p, q): h placed about the anchor, 0 elsewhere */
static double psf_hfine(const psf_geom* G, const double* h, int p, int q)
{
    const int ch = (G->Kh - 1) / 2;
    const int a = p - G->anchor + ch, b = q - G->anchor + ch;
    if (a < 0 || a >= G->Kh || b < 0 || b >= G->Kh) return 0.0;
    return h[a * G->Kh + b];
}

/* m = D(h * g) on f's stamp (Kf x Kf) */
static void psf_model(const psf_geom* G, const double* h, double* m)
{
    const int cg = (G->Kg - 1) / 2;
    for (int I = 0; I < G->Kf * G->Kf; ++I) m[I] = 0.0;
    for (int p = 0; p < G->S; ++p)
        for (int q = 0; q < G->S; ++q) {
            double c = 0.0;
            for (int i = 0; i < G->Kg; ++i)
                for (int j = 0; j < G->Kg; ++j)
                    c += G->g[i * G->Kg + j] * psf_hfine(G, h, p + cg - i, q + cg - j);
            m[(p / G->D) * G->Kf + q / G->D] += c;
        }
}

/* sum of squared forward differences of h extended by zeros */
static double psf_penalty(const psf_geom* G, const double* h)
{
    const int K = G->Kh;
    double s = 0.0;
    for (int i = -1; i < K; ++i)
        for (int j = -1; j < K; ++j) {
            const double c = (i >= 0 && j >= 0) ? h[i * K + j] : 0.0;
            if (j >= 0) {
                const double dn = (i + 1 < K) ? h[(i + 1) * K + j] : 0.0;
                if (i >= 0 || i + 1 < K) s += (dn - c) * (dn - c);
            }
            if (i >= 0) {
                const double rt = (j + 1 < K) ? h[i * K + j + 1] : 0.0;
                s += (rt - c) * (rt - c);
            }
        }
    return s;
}

static double psf_objective(const psf_geom* G, const float* f, double lambda, const double* h,
                            double* m)
{
    psf_model(G, h, m);
    double s = 0.0;
    for (int I = 0; I < G->Kf * G->Kf; ++I) {
        const double r = m[I] - (double)f[I];
        s += r * r;
    }
    return s + lambda * psf_penalty(G, h);
}

/* gradient of the objective with respect to h (Kh x Kh) */
static void psf_gradient(const psf_geom* G, const float* f, double lambda, const double* h,
                         double* m, double* grad)
{
    const int K = G->Kh, ch = (K - 1) / 2, cg = (G->Kg - 1) / 2;
    psf_model(G, h, m);
    for (int k = 0; k < K * K; ++k) grad[k] = 0.0;
    /* data term: 2 sum_{p,q} rho[p/D][q/D] * d(h*g)[p][q] / dh[a][b],
       (h*g)[p][q] = sum_{a,b} h[a][b] g[p + cg - (a - ch + anchor)][q + cg - (b - ch + anchor)] */
    for (int p = 0; p < G->S; ++p)
        for (int q = 0; q < G->S; ++q) {
            const double rho = m[(p / G->D) * G->Kf + q / G->D] - (double)f[(p / G->D) * G->Kf + q / G->D];
            for (int a = 0; a < K; ++a) {
                const int i = p + cg - (a - ch + G->anchor);
                if (i < 0 || i >= G->Kg) continue;
                for (int b = 0; b < K; ++b) {
                    const int j = q + cg - (b - ch + G->anchor);
                    if (j < 0 || j >= G->Kg) continue;
                    grad[a * K + b] += 2.0 * rho * G->g[i * G->Kg + j];
                }
            }
        }
    /* penalty: d/dh of lambda sum (differences)^2 = 2 lambda (4 h - sum of 4 neighbours) */
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            const double up = a > 0 ? h[(a - 1) * K + b] : 0.0;
            const double dn = a + 1 < K ? h[(a + 1) * K + b] : 0.0;
            const double lf = b > 0 ? h[a * K + b - 1] : 0.0;
            const double rt = b + 1 < K ? h[a * K + b + 1] : 0.0;
            grad[a * K + b] += 2.0 * lambda * (4.0 * h[a * K + b] - up - dn - lf - rt);
        }
}

static void psf_start(const psf_geom* G, const float* f, double* h)
{
    const int K = G->Kh, ch = (K - 1) / 2;
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
            const int p = a - ch + G->anchor, q = b - ch + G->anchor;
            double v = 0.0;
            if (p >= 0 && p < G->S && q >= 0 && q < G->S) {
                v = (double)f[(p / G->D) * G->Kf + q / G->D] / (double)(G->D * G->D);
                if (v < 0.0) v = 0.0;
            }
            h[a * K + b] = v;
        }
}

int em_oracle_psf_objective(int Kf, int Kh, int D, double sigma, double lambda, const float* f,
                            const double* h, double* model, double* objective)
{
    static psf_geom G;
    if (psf_geom_init(&G, Kf, Kh, D, sigma)) return -1;
    double* m = (double*)malloc(sizeof(double) * Kf * Kf);
    if (!m) return -2;
    *objective = psf_objective(&G, f, lambda, h, m);
    if (model) memcpy(model, m, sizeof(double) * Kf * Kf);
    free(m);
    return 0;
}

int em_oracle_psf_gradient(int Kf, int Kh, int D, double sigma, double lambda, const float* f,
                           const double* h, double* grad)
{
    static psf_geom G;
    if (psf_geom_init(&G, Kf, Kh, D, sigma)) return -1;
    double* m = (double*)malloc(sizeof(double) * Kf * Kf);
    if (!m) return -2;
    psf_gradient(&G, f, lambda, h, m, grad);
    free(m);
    return 0;
}

int em_oracle_psf_start(int Kf, int Kh, int D, const float* f, double* h)
{
    static psf_geom G;
    if (psf_geom_init(&G, Kf, Kh, D, 0.0)) return -1;
    psf_start(&G, f, h);
    return 0;
}

/* n independent fits of Eq. (4) by projected Adam (S steps each).  f: n x Kf x Kf
 * (binary32 data); h0: n x Kh x Kh or NULL (start of the header); h: n x Kh x Kh
 * result; objective: n values at the result, or NULL. */
int em_oracle_psf_fit(int n, int Kf, int Kh, int D, double sigma, double lambda, int S,
                      double lr, double decay, double beta1, double beta2, double eps,
                      const float* f, const float* h0, double* h, double* objective)
{
    static psf_geom G;
    if (psf_geom_init(&G, Kf, Kh, D, sigma) || n < 1 || S < 0) return -1;
    const int K2 = Kh * Kh;
    double* m = (double*)malloc(sizeof(double) * Kf * Kf);
    double* gr = (double*)malloc(sizeof(double) * K2);
    double* mo = (double*)malloc(sizeof(double) * K2);
    double* vo = (double*)malloc(sizeof(double) * K2);
    if (!m || !gr || !mo || !vo) { free(m); free(gr); free(mo); free(vo); return -2; }
    for (int t = 0; t < n; ++t) {
        const float* ft = f + (long)t * Kf * Kf;
        double* ht = h + (long)t * K2;
        if (h0) for (int k = 0; k < K2; ++k) ht[k] = (double)h0[(long)t * K2 + k];
        else psf_start(&G, ft, ht);
        double fmax = 0.0;
        for (int I = 0; I < Kf * Kf; ++I) if ((double)ft[I] > fmax) fmax = (double)ft[I];
        for (int k = 0; k < K2; ++k) { mo[k] = 0.0; vo[k] = 0.0; }
        for (int k = 1; k <= S; ++k) {
            psf_gradient(&G, ft, lambda, ht, m, gr);
            const double lrk = lr * fmax * pow(decay, S > 1 ? (double)(k - 1) / (double)(S - 1) : 0.0);
            const double c1 = 1.0 - pow(beta1, k), c2 = 1.0 - pow(beta2, k);
            for (int q = 0; q < K2; ++q) {
                mo[q] = beta1 * mo[q] + (1.0 - beta1) * gr[q];
                vo[q] = beta2 * vo[q] + (1.0 - beta2) * gr[q] * gr[q];
                const double step = lrk * (mo[q] / c1) / (sqrt(vo[q] / c2) + eps);
                const double nh = ht[q] - step;
                ht[q] = nh > 0.0 ? nh : 0.0;
            }
        }
        if (objective) objective[t] = psf_objective(&G, ft, lambda, ht, m);
    }
    free(m); free(gr); free(mo); free(vo);
    return 0;
}

/* ===========================================================================
 * Heavier-tailed noise (the robust model the paper names as future work in its
 * conclusion): each eta_t[i][j] of Eq. (1) is Student-t with nu degrees of
 * freedom and scale v_t[i][j] instead of Gaussian.  Written as a Gaussian
 * scale mixture (eta | w ~ N(0, v / w), w ~ Gamma(nu/2, rate nu/2); Lange,
 * Little & Taylor, 1989), the E-step gives each observed pixel the weight
 *     w = (nu + 1) / (nu + u (y - F x)^2)
 * at the current iterate, and the M-step is the update of Eq. (2) with u
 * replaced by u w (weights before the adjoint, clamp and guards as above):
 *     x <- x * max(B_w, 0) / Dn_w,   B_w = sum_t F_t^T(u_t w_t y_t),
 *                                    Dn_w = sum_t F_t^T(u_t w_t F_t x).
 * Unlike the Gaussian case the numerator changes every iteration.  The
 * log-likelihood is the Student-t one,
 *     l(x) = sum_t sum_{u>0} [ lgamma((nu+1)/2) - lgamma(nu/2) - ln(nu pi v)/2
 *                              - (nu+1)/2 ln(1 + u (y - F x)^2 / nu) ],
 * recorded before each update.
 * ========================================================================= */

static double emo_t_const(double nu)
{
    return lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) - 0.5 * log(nu * EMO_PI);
}

/* One pass at x: the weights w of every frame from F_t x, then B_w, Dn_w and l(x). */
static void emo_robust_terms(emo_state* st, double nu, const float* v, const double* x,
                             double* Bw, double* Dnw, double* loglik)
{
    const int Hl = st->Hf * st->sr, Wl = st->Wf * st->sr;
    const double cnu = emo_t_const(nu);
    double ll = 0.0;
    double* rb = (double*)malloc(sizeof(double) * st->nf);
    for (long j = 0; j < st->nl; ++j) { Bw[j] = 0.0; Dnw[j] = 0.0; }
    for (int t = 0; t < st->n; ++t) {
        const double* ft = st->f + (long)t * st->K * st->K;
        const double* ut = st->u + (long)t * st->nf;
        const double* yt = st->yh + (long)t * st->nf;
        em_oracle_forward(st->K, st->sr, Hl, Wl, ft, x, st->m);
        for (long p = 0; p < st->nf; ++p) {
            if (ut[p] > 0.0) {
                const double d = yt[p] - st->m[p];
                const double z = ut[p] * d * d;
                const double w = (nu + 1.0) / (nu + z);
                st->r[p] = ut[p] * w * st->m[p];
                rb[p] = ut[p] * w * yt[p];
                ll += cnu - 0.5 * log((double)v[(long)t * st->nf + p]) - 0.5 * (nu + 1.0) * log1p(z / nu);
            } else {
                st->r[p] = 0.0;
                rb[p] = 0.0;
            }
        }
        em_oracle_adjoint(st->K, st->sr, Hl, Wl, ft, st->r, st->s);
        for (long j = 0; j < st->nl; ++j) Dnw[j] += st->s[j];
        em_oracle_adjoint(st->K, st->sr, Hl, Wl, ft, rb, st->s);
        for (long j = 0; j < st->nl; ++j) Bw[j] += st->s[j];
    }
    free(rb);
    if (loglik) *loglik = ll;
}

/* Student-t l(x). */
int em_oracle_loglik_t(int n, int Hf, int Wf, int K, int sr, double nu,
                       const float* y, const float* v, const float* psf,
                       const double* x, double* out)
{
    if (!(nu > 0.0)) return -1;
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    double* B = (double*)malloc(sizeof(double) * st.nl);
    double* D = (double*)malloc(sizeof(double) * st.nl);
    if (!B || !D) { free(B); free(D); emo_free(&st); return -2; }
    emo_robust_terms(&st, nu, v, x, B, D, out);
    free(B); free(D);
    emo_free(&st);
    return 0;
}

/* B_w and Dn_w at x (latent grid each). */
int em_oracle_terms_t(int n, int Hf, int Wf, int K, int sr, double nu,
                      const float* y, const float* v, const float* psf,
                      const double* x, double* Bw, double* Dnw)
{
    if (!(nu > 0.0)) return -1;
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    emo_robust_terms(&st, nu, v, x, Bw, Dnw, NULL);
    emo_free(&st);
    return 0;
}

/* k_max iterations of the Student-t EM from x (in: x^(0), out: x^(k_max));
 * trace[k-1] = l(x^(k-1)) (Student-t), relchange as em_oracle_run. */
int em_oracle_run_t(int n, int Hf, int Wf, int K, int sr, double nu,
                    const float* y, const float* v, const float* psf,
                    double* x, int k_max, double* trace, double* relchange)
{
    if (n < 1 || Hf < 1 || Wf < 1 || K < 1 || (K % 2) == 0 || (sr != 1 && sr != 2)) return -1;
    if (!(nu > 0.0)) return -1;
    emo_state st;
    if (emo_setup(&st, n, Hf, Wf, K, sr, y, v, psf)) return -2;
    if (st.bad) { emo_free(&st); return -1; }
    double* B = (double*)malloc(sizeof(double) * st.nl);
    double* Dn = (double*)malloc(sizeof(double) * st.nl);
    if (!B || !Dn) { free(B); free(Dn); emo_free(&st); return -2; }
    for (int k = 1; k <= k_max; ++k) {
        double ll = 0.0, a = 0.0, b = 0.0;
        emo_robust_terms(&st, nu, v, x, B, Dn, &ll);
        if (trace) trace[k - 1] = ll;
        emo_update(st.nl, B, Dn, x, &a, &b);
        if (relchange) relchange[k - 1] = b > 0.0 ? sqrt(a) / sqrt(b) : 0.0;
    }
    free(B); free(Dn);
    emo_free(&st);
    return 0;
}
