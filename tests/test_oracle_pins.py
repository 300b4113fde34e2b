"""Pins of the FP64 oracle against what the paper and mathematics fix.

Every check here is independent of the oracle's own code path: closed forms,
dense matrices built from the operator definition, scipy library routines,
invariants stated in the paper (Sec. 2) and optimality conditions.  A plausible
mistake in the oracle (dropped term, wrong sign, wrong index, transposed
operand, wrong guard) breaks at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.signal

import oracle
from paper_2302_05804_amd import synth

RNG = np.random.default_rng


# ---------------------------------------------------------------------------
# helpers written from the definitions (not from the oracle)
# ---------------------------------------------------------------------------

def dense_H(f, H, W):
    """Dense matrix of the zero-filled 'same' convolution x -> f * x (Eq. (1))."""
    K = f.shape[0]
    c = (K - 1) // 2
    M = np.zeros((H * W, H * W))
    for i in range(H):
        for j in range(W):
            for k in range(H):
                for l in range(W):
                    a, b = i - k + c, j - l + c
                    if 0 <= a < K and 0 <= b < K:
                        M[i * W + j, k * W + l] = f[a, b]
    return M


def dense_D(Hl, Wl):
    """Dense 2x2 box-sum downsampler (Eq. (3)), latent -> frame grid."""
    Hf, Wf = Hl // 2, Wl // 2
    M = np.zeros((Hf * Wf, Hl * Wl))
    for i in range(Hl):
        for j in range(Wl):
            M[(i // 2) * Wf + j // 2, i * Wl + j] = 1.0
    return M


def dense_F(f, Hl, Wl, sr):
    Hm = dense_H(np.asarray(f, np.float64), Hl, Wl)
    return Hm if sr == 1 else dense_D(Hl, Wl) @ Hm


def small_problem(Hl, Wl, n, K, sr=1, seed=0, mask=0.0, sky=(20.0, 60.0)):
    """A small random problem (inputs only), positive PSFs and variances."""
    rng = RNG(seed)
    Hf, Wf = Hl // sr, Wl // sr
    psf = rng.uniform(0.05, 1.0, (n, K, K)).astype(np.float32)
    psf /= psf.sum(axis=(1, 2), keepdims=True)
    x_true = rng.gamma(1.0, 50.0, (Hl, Wl))
    y = np.empty((n, Hf, Wf), np.float32)
    v = np.empty((n, Hf, Wf), np.float32)
    for t in range(n):
        mdl = dense_F(psf[t], Hl, Wl, sr) @ x_true.ravel()
        var = rng.uniform(*sky) + mdl
        y[t] = (mdl + np.sqrt(var) * rng.standard_normal(mdl.size)).reshape(Hf, Wf)
        v[t] = var.reshape(Hf, Wf)
        if mask > 0:
            mk = rng.uniform(size=(Hf, Wf)) < mask
            y[t][mk] = np.nan
            v[t][mk] = np.inf
    return y, v, psf, x_true


def positive(shape, seed, lo=1.0, hi=100.0):
    return RNG(seed).uniform(lo, hi, shape).astype(np.float32)


# ---------------------------------------------------------------------------
# P4: operators equal the library's convolve2d / correlate2d; adjoint test
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K,H,W", [(3, 9, 7), (15, 20, 33), (43, 50, 47), (5, 1, 1), (7, 3, 11)])
def test_forward_is_convolve2d_same(K, H, W):
    rng = RNG(K * 100 + H)
    f = rng.uniform(-1, 1, (K, K))
    x = rng.uniform(-1, 1, (H, W))
    m = oracle.forward(f, x, sr=1)
    ref = scipy.signal.convolve2d(x, f, mode="same")
    np.testing.assert_allclose(m, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("K,H,W", [(3, 9, 7), (15, 20, 33), (43, 50, 47), (7, 3, 11)])
def test_adjoint_is_correlate2d_same(K, H, W):
    rng = RNG(K * 7 + W)
    f = rng.uniform(-1, 1, (K, K))
    r = rng.uniform(-1, 1, (H, W))
    s = oracle.adjoint(f, r, sr=1)
    ref = scipy.signal.correlate2d(r, f, mode="same")
    np.testing.assert_allclose(s, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("sr", [1, 2])
@pytest.mark.parametrize("K,Hl,Wl", [(5, 12, 10), (15, 34, 22), (43, 60, 52)])
def test_adjoint_dot_product(sr, K, Hl, Wl):
    rng = RNG(K + 31 * sr)
    f = rng.uniform(0, 1, (K, K))
    x = rng.uniform(-1, 1, (Hl, Wl))
    r = rng.uniform(-1, 1, (Hl // sr, Wl // sr))
    lhs = np.vdot(oracle.forward(f, x, sr), r)
    rhs = np.vdot(x, oracle.adjoint(f, r, sr))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.abs(x).sum() * np.abs(r).sum() / x.size)


def test_sr2_forward_is_box_sum_of_same_conv():
    rng = RNG(5)
    f = rng.uniform(0, 1, (7, 7))
    x = rng.uniform(0, 1, (18, 14))
    z = scipy.signal.convolve2d(x, f, mode="same")
    ref = z.reshape(9, 2, 7, 2).sum(axis=(1, 3))
    np.testing.assert_allclose(oracle.forward(f, x, sr=2), ref, rtol=0, atol=1e-12)


def test_sr2_adjoint_is_correlate_of_replicated():
    rng = RNG(6)
    f = rng.uniform(0, 1, (9, 9))
    r = rng.uniform(-1, 1, (8, 11))
    up = np.repeat(np.repeat(r, 2, axis=0), 2, axis=1)
    ref = scipy.signal.correlate2d(up, f, mode="same")
    np.testing.assert_allclose(oracle.adjoint(f, r, sr=2), ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# P3: dense brute force on 8x8 images (explicit F_t matrices)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sr,mask", [(1, 0.0), (1, 0.15), (2, 0.0), (2, 0.15)])
def test_dense_8x8_operators_loglik_and_step(sr, mask):
    Hl = Wl = 8
    n, K = 3, 5
    y, v, psf, _ = small_problem(Hl, Wl, n, K, sr=sr, seed=11 + sr, mask=mask)
    x0 = positive((Hl, Wl), 3)
    Fs = [dense_F(psf[t], Hl, Wl, sr) for t in range(n)]
    masked = ~np.isfinite(v)
    u = np.where(masked, 0.0, 1.0 / v.astype(np.float64))
    yh = np.where(masked, 0.0, y.astype(np.float64))
    xv = x0.astype(np.float64).ravel()
    # operators
    for t in range(n):
        np.testing.assert_allclose(oracle.forward(psf[t], x0, sr).ravel(), Fs[t] @ xv,
                                   rtol=1e-13, atol=1e-12)
        r = RNG(t).uniform(-1, 1, Fs[t].shape[0])
        np.testing.assert_allclose(
            oracle.adjoint(psf[t], r.reshape(Hl // sr, Wl // sr), sr).ravel(), Fs[t].T @ r,
            rtol=1e-13, atol=1e-13)
    # log-likelihood of Eq. (1)
    ll = 0.0
    for t in range(n):
        uu, yy, vv = u[t].ravel(), yh[t].ravel(), v[t].astype(np.float64).ravel()
        res = yy - Fs[t] @ xv
        keep = uu > 0
        ll += -0.5 * np.sum(uu[keep] * res[keep] ** 2 + np.log(2 * np.pi * vv[keep]))
    assert oracle.loglik(y, v, psf, x0, sr) == pytest.approx(ll, rel=1e-13)
    # one EM step of Eq. (2), weights applied on the frame grid before F^T
    B = sum(Fs[t].T @ (u[t].ravel() * yh[t].ravel()) for t in range(n))
    Dn = sum(Fs[t].T @ (u[t].ravel() * (Fs[t] @ xv)) for t in range(n))
    x1 = xv * np.maximum(B, 0) / Dn
    np.testing.assert_allclose(oracle.numerator(y, v, psf, sr).ravel(), B, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.denominator(y, v, psf, x0, sr).ravel(), Dn, rtol=1e-12)
    np.testing.assert_allclose(oracle.run(y, v, psf, x0, 1, sr).ravel(), x1, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("sr", [1, 2])
def test_dense_8x8_monotone_towards_nnls_optimum(sr):
    """When B > 0 everywhere, the EM iterates never pass the likelihood of the
    constrained optimum (NNLS of the stacked sqrt(u) F x ~ sqrt(u) y) and approach it."""
    Hl = Wl = 8
    n, K = 4, 3
    # bright, noise-light data so that B > 0 everywhere
    y, v, psf, xt = small_problem(Hl, Wl, n, K, sr=sr, seed=21 + sr, sky=(1.0, 2.0))
    B = oracle.numerator(y, v, psf, sr)
    assert (B > 0).all()
    Fs = [dense_F(psf[t], Hl, Wl, sr) for t in range(n)]
    u = 1.0 / v.astype(np.float64)
    A = np.vstack([np.sqrt(u[t].ravel())[:, None] * Fs[t] for t in range(n)])
    b = np.concatenate([np.sqrt(u[t].ravel()) * y[t].astype(np.float64).ravel() for t in range(n)])
    xopt, _ = scipy.optimize.nnls(A, b, maxiter=50 * A.shape[1])
    ll_opt = oracle.loglik(y, v, psf, xopt.reshape(Hl, Wl), sr)
    x0 = np.full((Hl, Wl), oracle.flat_x0(y, v, sr), np.float32)
    lls = []
    x = x0.astype(np.float64)
    for k in (10, 100, 1000, 5000):
        x = oracle.run(y, v, psf, x0, k, sr)
        lls.append(oracle.loglik(y, v, psf, x, sr))
    assert all(l <= ll_opt + 1e-9 * abs(ll_opt) for l in lls)
    assert all(b2 >= a2 - 1e-9 * abs(a2) for a2, b2 in zip(lls, lls[1:]))
    gap0 = ll_opt - oracle.loglik(y, v, psf, x0, sr)
    assert ll_opt - lls[-1] < 1e-3 * gap0


# ---------------------------------------------------------------------------
# P1 / P2: delta PSFs give the inverse-variance-weighted mean in closed form
# ---------------------------------------------------------------------------

def test_delta_psf_gives_weighted_mean_sr1():
    n, H, W, K = 5, 13, 11, 7
    rng = RNG(1)
    psf = np.zeros((n, K, K), np.float32)
    psf[:, K // 2, K // 2] = 1.0
    y = rng.normal(30, 40, (n, H, W)).astype(np.float32)   # some negative means
    v = rng.uniform(5, 50, (n, H, W)).astype(np.float32)
    mk = rng.uniform(size=(n, H, W)) < 0.2
    mk[:, 0, 0] = True                                      # one pixel masked in every frame
    y[mk] = np.nan
    v[mk] = np.inf
    x0 = positive((H, W), 9)
    u = np.where(mk, 0.0, 1.0 / v.astype(np.float64))
    yy = np.where(mk, 0.0, y.astype(np.float64))
    su = u.sum(0)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = (u * yy).sum(0) / su
    expect = np.where(su > 0, np.maximum(mean, 0.0), x0.astype(np.float64))
    x1 = oracle.run(y, v, psf, x0, 1)
    np.testing.assert_allclose(x1, expect, rtol=1e-13, atol=1e-300)
    assert x1[0, 0] == x0[0, 0]                             # unobserved pixel keeps its value
    x7 = oracle.run(y, v, psf, x0, 7)                        # and it is a fixed point
    np.testing.assert_allclose(x7, expect, rtol=1e-13, atol=1e-300)


def test_delta_psf_sr2_block_sums_and_proportions():
    n, Hf, Wf, K = 4, 6, 5, 5
    rng = RNG(2)
    psf = np.zeros((n, K, K), np.float32)
    psf[:, K // 2, K // 2] = 1.0
    y = rng.normal(20, 30, (n, Hf, Wf)).astype(np.float32)
    v = rng.uniform(5, 50, (n, Hf, Wf)).astype(np.float32)
    x0 = positive((2 * Hf, 2 * Wf), 4)
    u = 1.0 / v.astype(np.float64)
    mean = (u * y).sum(0) / u.sum(0)
    x1 = oracle.run(y, v, psf, x0, 1, sr=2)
    blocks = x1.reshape(Hf, 2, Wf, 2).sum(axis=(1, 3))
    np.testing.assert_allclose(blocks, np.maximum(mean, 0.0), rtol=1e-13, atol=1e-12)
    x0b = x0.astype(np.float64).reshape(Hf, 2, Wf, 2)
    prop0 = x0b / x0b.sum(axis=(1, 3), keepdims=True)
    x1b = x1.reshape(Hf, 2, Wf, 2)
    pos = (mean > 0)[:, None, :, None] * np.ones_like(x1b, bool)
    prop1 = x1b / np.where(pos, x1b.sum(axis=(1, 3), keepdims=True), 1.0)
    np.testing.assert_allclose(prop1[pos], prop0[pos], rtol=1e-13)


# ---------------------------------------------------------------------------
# P5 / P6: monotone log-likelihood, non-negative iterates (Sec. 2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sr,mask", [(1, 0.0), (1, 0.05), (2, 0.05)])
def test_loglik_monotone_and_nonnegative(sr, mask):
    y, v, psf, _ = small_problem(24, 20, 3, 7, sr=sr, seed=31 + sr, mask=mask)
    x0 = positive((24, 20), 5)
    x, tr, _ = oracle.run(y, v, psf, x0, 60, sr, trace=True)
    assert (np.diff(tr) >= -1e-12 * np.abs(tr[1:])).all()
    assert (x >= 0).all()
    # the trace entries are l(x^(k-1))
    assert tr[0] == pytest.approx(oracle.loglik(y, v, psf, x0, sr), rel=1e-14)


def test_c1_workload_monotone_nonnegative():
    p = synth.make_problem("c1")
    x0 = np.full(p.latent_shape, oracle.flat_x0(p.y, p.v), np.float32)
    x, tr, rc = oracle.run(p.y, p.v, p.psf, x0, 10, trace=True, relchange=True)
    assert (np.diff(tr) >= -1e-12 * np.abs(tr[1:])).all()
    assert (x >= 0).all() and (rc > 0).all()


# ---------------------------------------------------------------------------
# P7: noise-free data generated by a strictly positive sky is a fixed point
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sr", [1, 2])
def test_noise_free_fixed_point(sr):
    Hl, Wl, n, K = 16, 14, 3, 5
    rng = RNG(40 + sr)
    psf = rng.uniform(0.1, 1, (n, K, K)).astype(np.float32)
    xs = rng.uniform(1, 10, (Hl, Wl))
    y = np.stack([dense_F(psf[t], Hl, Wl, sr) @ xs.ravel() for t in range(n)])
    y = y.reshape(n, Hl // sr, Wl // sr)
    # y must be representable exactly in FP32 for the fixed point to be exact:
    # re-derive xs so that F xs is what the oracle sees (it widens y from float).
    v = rng.uniform(1, 3, y.shape).astype(np.float32)
    y32 = y.astype(np.float32)
    x1 = oracle.run(y32, v, psf, xs.astype(np.float32), 1, sr)
    np.testing.assert_allclose(x1, xs.astype(np.float32).astype(np.float64), rtol=2e-6)


# ---------------------------------------------------------------------------
# P8 / P9: order independence and invariances (Sec. 2)
# ---------------------------------------------------------------------------

def test_frame_permutation_invariance():
    y, v, psf, _ = small_problem(20, 18, 5, 7, seed=50, mask=0.05)
    x0 = positive((20, 18), 6)
    perm = [3, 0, 4, 1, 2]
    a = oracle.run(y, v, psf, x0, 15)
    b = oracle.run(y[perm], v[perm], psf[perm], x0, 15)
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-11 * a.max())


def test_invariances():
    y, v, psf, _ = small_problem(18, 16, 3, 5, seed=60, mask=0.1)
    x0 = positive((18, 16), 7)
    base = oracle.run(y, v, psf, x0, 12)
    # scaling all variances
    np.testing.assert_allclose(oracle.run(y, v * np.float32(4.0), psf, x0, 12), base,
                               rtol=1e-11, atol=1e-11 * base.max())
    # duplicating every frame
    np.testing.assert_allclose(oracle.run(np.concatenate([y, y]), np.concatenate([v, v]),
                                          np.concatenate([psf, psf]), x0, 12), base,
                               rtol=1e-11, atol=1e-11 * base.max())
    # scaling y and x0 together (powers of two keep the inputs exact)
    np.testing.assert_allclose(oracle.run(y * np.float32(8.0), v, psf, x0 * np.float32(8.0), 12),
                               8.0 * base, rtol=1e-11, atol=1e-11 * base.max())
    # values of y at masked pixels do not matter at all
    y2 = y.copy()
    y2[~np.isfinite(v)] = 1e30
    assert np.array_equal(oracle.run(y2, v, psf, x0, 12), base)


# ---------------------------------------------------------------------------
# P10: KKT conditions of the constrained MLE after many iterations
# ---------------------------------------------------------------------------

def test_kkt_at_convergence():
    y, v, psf, _ = small_problem(10, 10, 3, 3, seed=70, sky=(5.0, 10.0))
    x0 = np.full((10, 10), oracle.flat_x0(y, v), np.float32)
    x = oracle.run(y, v, psf, x0, 10000)
    B = oracle.numerator(y, v, psf)
    Dn = oracle.denominator(y, v, psf, x)
    act = x > 1e-3 * x.max()
    np.testing.assert_allclose(B[act], Dn[act], rtol=1e-4)
    assert (B[~act] <= Dn[~act] * (1 + 1e-4) + 1e-12).all()


# ---------------------------------------------------------------------------
# P11: the as-typeset weighting equals the adjoint weighting for constant v_t
# ---------------------------------------------------------------------------

def test_literal_equals_adjoint_for_constant_variance():
    y, _, psf, _ = small_problem(16, 16, 3, 5, seed=80)
    v = np.stack([np.full((16, 16), s, np.float32) for s in (7.0, 21.0, 40.0)])
    x0 = positive((16, 16), 8)
    a = oracle.run(y, v, psf, x0, 10, mode=oracle.W_ADJOINT)
    b = oracle.run(y, v, psf, x0, 10, mode=oracle.W_LITERAL)
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-11 * a.max())


@pytest.mark.parametrize("shape", [(8, 8), (8, 6)])
def test_literal_weighting_dense_spatially_varying(shape):
    """Eq. (2) as typeset, with u varying over pixels and masked: from explicit
    F_t matrices, B = sum_t u_t (.) (F_t^T yhat_t) and
    Dn = sum_t u_t (.) (F_t^T F_t x), u read on the latent grid (= frame grid,
    sr = 1) at the same pixel as the adjoint's output.  A non-square grid and
    per-pixel random u make a transposed, shifted or frame-swapped read of u
    fail; so does weighting before the adjoint."""
    Hl, Wl = shape
    n, K = 3, 5
    y, v, psf, _ = small_problem(Hl, Wl, n, K, seed=82, mask=0.15, sky=(5.0, 300.0))
    rng = RNG(83)
    # spread v over two decades so that u differs strongly between pixels
    v = np.where(np.isinf(v), v, v * rng.uniform(0.1, 10.0, v.shape)).astype(np.float32)
    v64 = v.astype(np.float64)
    u = np.where(np.isinf(v64), 0.0, 1.0 / v64)
    yh = np.where(u > 0, y.astype(np.float64), 0.0)
    x = positive((Hl, Wl), 84)
    Fs = [dense_F(psf[t], Hl, Wl, 1) for t in range(n)]
    B = sum(u[t].ravel() * (Fs[t].T @ yh[t].ravel()) for t in range(n)).reshape(Hl, Wl)
    Dn = sum(u[t].ravel() * (Fs[t].T @ (Fs[t] @ x.ravel().astype(np.float64)))
             for t in range(n)).reshape(Hl, Wl)
    Bo = oracle.numerator(y, v, psf, mode=oracle.W_LITERAL)
    Dno = oracle.denominator(y, v, psf, x, mode=oracle.W_LITERAL)
    np.testing.assert_allclose(Bo, B, rtol=1e-12, atol=1e-12 * np.abs(B).max())
    np.testing.assert_allclose(Dno, Dn, rtol=1e-12, atol=1e-12 * np.abs(Dn).max())
    # one step of the typeset update, with the clamp and guards
    x64 = x.astype(np.float64)
    x1 = np.where(Dn == 0, x64, x64 * np.maximum(B, 0.0) / np.where(Dn == 0, 1.0, Dn))
    xo = oracle.run(y, v, psf, x, 1, mode=oracle.W_LITERAL)
    np.testing.assert_allclose(xo, x1, rtol=1e-12, atol=1e-12 * x1.max())
    # the two weightings really differ here, so the pin tells them apart
    Ba = oracle.numerator(y, v, psf, mode=oracle.W_ADJOINT)
    assert np.abs(Ba - B).max() > 1e-3 * np.abs(B).max()


def test_literal_differs_for_varying_variance():
    y, v, psf, _ = small_problem(16, 16, 3, 5, seed=81, mask=0.1)
    x0 = positive((16, 16), 8)
    a = oracle.run(y, v, psf, x0, 3, mode=oracle.W_ADJOINT)
    b = oracle.run(y, v, psf, x0, 3, mode=oracle.W_LITERAL)
    assert np.abs(a - b).max() > 1e-6 * a.max()


# ---------------------------------------------------------------------------
# flat starting guess and the point-wise step
# ---------------------------------------------------------------------------

def test_flat_x0_closed_form():
    rng = RNG(90)
    y = rng.normal(5, 2, (3, 7, 6)).astype(np.float32)
    v = rng.uniform(1, 4, (3, 7, 6)).astype(np.float32)
    v[0, 1, 2] = np.inf
    y[0, 1, 2] = np.nan
    ok = np.isfinite(v)
    mu = (y[ok].astype(np.float64) / v[ok]).sum() / (1.0 / v[ok].astype(np.float64)).sum()
    assert oracle.flat_x0(y, v, 1) == pytest.approx(mu, rel=1e-14)
    assert oracle.flat_x0(y, v, 2) == pytest.approx(mu / 4, rel=1e-14)
    assert oracle.flat_x0(-np.abs(y), v, 1) == pytest.approx(1e-3, rel=1e-14)


@pytest.mark.parametrize("sr", [1, 2])
def test_step_at_matches_dense_step(sr):
    Hl, Wl, n, K = 12, 10, 2, 5
    y, v, psf, _ = small_problem(Hl, Wl, n, K, sr=sr, seed=95 + sr, mask=0.1)
    x0 = positive((Hl, Wl), 10)
    Fs = [dense_F(psf[t], Hl, Wl, sr) for t in range(n)]
    masked = ~np.isfinite(v)
    u = np.where(masked, 0.0, 1.0 / v.astype(np.float64))
    yh = np.where(masked, 0.0, y.astype(np.float64))
    xv = x0.astype(np.float64).ravel()
    B = sum(Fs[t].T @ (u[t].ravel() * yh[t].ravel()) for t in range(n))
    Dn = sum(Fs[t].T @ (u[t].ravel() * (Fs[t] @ xv)) for t in range(n))
    x1 = xv * np.maximum(B, 0) / Dn
    rows = np.array([0, 3, 11, 5, 7])
    cols = np.array([0, 9, 4, 5, 1])
    Bp, Dp, xp = oracle.step_at(y, v, psf, x0, rows, cols, sr)
    idx = rows * Wl + cols
    np.testing.assert_allclose(Bp, B[idx], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(Dp, Dn[idx], rtol=1e-12)
    np.testing.assert_allclose(xp, x1[idx], rtol=1e-12, atol=1e-14)


def test_invalid_inputs_rejected():
    y, v, psf, _ = small_problem(8, 8, 2, 3, seed=99)
    x0 = positive((8, 8), 1)
    for bad in (0.0, -1.0, np.nan, -np.inf):
        vb = v.copy()
        vb[1, 2, 3] = bad
        with pytest.raises(ValueError):
            oracle.run(y, vb, psf, x0, 1)
    yb = y.copy()
    yb[0, 0, 0] = np.nan
    with pytest.raises(ValueError):
        oracle.run(yb, v, psf, x0, 1)


# ---------------------------------------------------------------------------
# The super-resolution run the paper describes after Eq. (4): exposures
# up-sampled to the fine grid (reading: flux-sharing replication), plain EM
# with the super-resolved PSFs, no D.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("D", [2, 3, 4])
def test_upsample_is_flux_sharing_replication(D):
    rng = RNG(40 + D)
    y = rng.normal(10, 30, (3, 5, 7)).astype(np.float32)
    v = rng.uniform(1, 50, (3, 5, 7)).astype(np.float32)
    v[1, 2, 3] = np.inf
    y[1, 2, 3] = np.nan
    yd, vd = oracle.upsample(y, v, D)
    rep = lambda a: np.repeat(np.repeat(a, D, axis=1), D, axis=2)
    assert np.array_equal(yd, rep(y) / np.float32(D * D), equal_nan=True)
    assert np.array_equal(vd, rep(v) / np.float32(D ** 4))
    assert np.isinf(vd[1, 2 * D:3 * D, 3 * D:4 * D]).all()
    # the D x D block sums give the frame back (exactly for powers of two)
    ok = np.isfinite(y)
    bs = yd.astype(np.float64).reshape(3, 5, D, 7, D).sum(axis=(2, 4))
    np.testing.assert_allclose(bs[ok], y[ok], rtol=0 if D in (2, 4) else 1e-6, atol=0)
    with pytest.raises(ValueError):
        oracle.upsample(y, v, 5)


def test_upsampled_delta_psf_gives_scaled_weighted_mean():
    """With a delta PSF on the fine grid one update gives, in every fine pixel,
    the inverse-variance-weighted mean of the frames divided by D^2."""
    D, n, H, W = 2, 4, 6, 5
    rng = RNG(44)
    y = rng.normal(20, 30, (n, H, W)).astype(np.float32)
    v = rng.uniform(5, 50, (n, H, W)).astype(np.float32)
    mk = rng.uniform(size=(n, H, W)) < 0.2
    y[mk] = np.nan
    v[mk] = np.inf
    yd, vd = oracle.upsample(y, v, D)
    h = np.ones((n, 1, 1), np.float32)
    x0 = positive((D * H, D * W), 45)
    u = np.where(mk, 0.0, 1.0 / v.astype(np.float64))
    su = u.sum(0)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = (u * np.where(mk, 0.0, y.astype(np.float64))).sum(0) / su
    coarse = np.where(su > 0, np.maximum(mean, 0.0) / (D * D), np.nan)
    fine = np.repeat(np.repeat(coarse, D, 0), D, 1)
    fine = np.where(np.isnan(fine), x0.astype(np.float64), fine)
    x1 = oracle.run(yd, vd, h, x0, 1)
    np.testing.assert_allclose(x1, fine, rtol=1e-12, atol=1e-300)


def test_upsampled_run_ignores_variance_factor():
    """The D^4 factor of v^D scales every weight by the same constant, which
    leaves the iterates unchanged (P9); only the value of l moves."""
    D = 2
    y, v, _, _ = small_problem(8, 6, 3, 3, seed=46, mask=0.1)
    hd = RNG(47).uniform(0.05, 1.0, (3, 7, 7)).astype(np.float32)
    hd /= hd.sum(axis=(1, 2), keepdims=True)
    yd, vd = oracle.upsample(y, v, D)
    vr = np.repeat(np.repeat(v, D, axis=1), D, axis=2)
    x0 = positive((16, 12), 48)
    a = oracle.run(yd, vd, hd, x0, 6)
    b = oracle.run(yd, vr, hd, x0, 6)
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-12 * np.abs(a).max())
