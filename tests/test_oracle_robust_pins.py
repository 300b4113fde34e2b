"""Pins of the oracle's Student-t EM (heavier-tailed noise, the robust model the
paper names as future work): the log-likelihood against scipy.stats.t, the
Gaussian limit nu -> infinity, one step against dense matrices built from the
operator definitions, the delta-PSF closed form, monotone likelihood (the
step is a minorise-maximise step of the Student-t likelihood), a scaling
invariance, and the down-weighting of outliers.
"""
import numpy as np
import pytest
import scipy.stats

import oracle
from tests.test_oracle_pins import RNG, dense_F, positive, small_problem


def with_outliers(y, v, frac, amp, seed):
    """Unmasked outliers (e.g. a satellite trail): +amp * sqrt(v) at a fraction of pixels."""
    rng = RNG(seed)
    y = y.copy()
    hit = (rng.uniform(size=y.shape) < frac) & np.isfinite(v)
    y[hit] += (amp * np.sqrt(v[hit])).astype(np.float32)
    return y, hit


@pytest.mark.parametrize("sr", [1, 2])
def test_loglik_is_scipy_student_t(sr):
    y, v, psf, _ = small_problem(12, 10, 3, 5, sr=sr, seed=71, mask=0.1)
    x = positive((12, 10), 72)
    nu = 3.5
    ref = 0.0
    for t in range(3):
        m = (dense_F(psf[t], 12, 10, sr) @ x.astype(np.float64).ravel()).reshape(y.shape[1:])
        ok = np.isfinite(v[t])
        ref += scipy.stats.t.logpdf(y[t][ok].astype(np.float64), df=nu, loc=m[ok],
                                    scale=np.sqrt(v[t][ok].astype(np.float64))).sum()
    got = oracle.loglik_t(y, v, psf, x, nu, sr)
    assert abs(got - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("sr", [1, 2])
def test_gaussian_limit(sr):
    """nu -> infinity: the weights tend to 1 and the iteration to Eq. (2); the
    log-likelihood tends to the Gaussian one (compared at nu = 1e9: the model
    difference is about sum z^2 / (4 nu) with z = u (y - F x)^2 up to ~100
    here, and lgamma's cancellation costs ~1e-6 per pixel)."""
    y, v, psf, _ = small_problem(10, 12, 3, 5, sr=sr, seed=73, mask=0.05)
    x0 = positive((10, 12), 74)
    a = oracle.run_t(y, v, psf, x0, 6, 1e12, sr)
    b, trb, _ = oracle.run(y, v, psf, x0, 6, sr, trace=True)
    np.testing.assert_allclose(a, b, rtol=1e-8, atol=1e-10 * np.abs(b).max())
    _, tra, _ = oracle.run_t(y, v, psf, x0, 6, 1e9, sr, trace=True)
    np.testing.assert_allclose(tra, trb, rtol=1e-6)


@pytest.mark.parametrize("sr", [1, 2])
def test_one_step_matches_dense_matrices(sr):
    Hl, Wl, n, nu = 8, 8, 3, 2.5
    y, v, psf, _ = small_problem(Hl, Wl, n, 3, sr=sr, seed=75, mask=0.1)
    y, _ = with_outliers(y, v, 0.05, 40.0, 76)
    x0 = positive((Hl, Wl), 77).astype(np.float64)
    B = np.zeros(Hl * Wl)
    D = np.zeros(Hl * Wl)
    for t in range(n):
        F = dense_F(psf[t], Hl, Wl, sr)
        m = F @ x0.ravel()
        ok = np.isfinite(v[t].ravel())
        u = np.where(ok, 1.0 / v[t].ravel().astype(np.float64), 0.0)
        yy = np.where(ok, y[t].ravel().astype(np.float64), 0.0)
        w = (nu + 1.0) / (nu + u * (yy - m) ** 2)
        B += F.T @ (u * w * yy)
        D += F.T @ (u * w * m)
    Bo, Do = oracle.terms_t(y, v, psf, x0, nu, sr)
    np.testing.assert_allclose(Bo.ravel(), B, rtol=1e-12, atol=1e-12 * np.abs(B).max())
    np.testing.assert_allclose(Do.ravel(), D, rtol=1e-12, atol=1e-12 * np.abs(D).max())
    x1 = np.where(D > 0, x0.ravel() * np.maximum(B, 0) / np.where(D > 0, D, 1), x0.ravel())
    got = oracle.run_t(y, v, psf, x0, 1, nu, sr)
    np.testing.assert_allclose(got.ravel(), x1, rtol=1e-12, atol=1e-12 * np.abs(x1).max())


def test_delta_psf_one_step_is_weighted_mean():
    """f = impulse: x1 = max(0, sum_t u w y / sum_t u w) per pixel, w from x0."""
    n, H, W, nu = 5, 6, 7, 3.0
    rng = RNG(78)
    y = rng.normal(30, 10, (n, H, W)).astype(np.float32)
    v = rng.uniform(5, 50, (n, H, W)).astype(np.float32)
    y[1, 2, 3] = 5000.0                                   # an outlier
    psf = np.ones((n, 1, 1), np.float32)
    x0 = positive((H, W), 79).astype(np.float64)
    u = 1.0 / v.astype(np.float64)
    w = (nu + 1) / (nu + u * (y.astype(np.float64) - x0[None]) ** 2)
    ref = np.maximum(0, (u * w * y).sum(0) / (u * w).sum(0))
    got = oracle.run_t(y, v, psf, x0, 1, nu)
    np.testing.assert_allclose(got, ref, rtol=1e-13)


@pytest.mark.parametrize("sr,nu", [(1, 1.0), (1, 4.0), (2, 2.0)])
def test_loglik_is_monotone(sr, nu):
    y, v, psf, _ = small_problem(16, 14, 3, 5, sr=sr, seed=80 + sr, mask=0.05)
    y, _ = with_outliers(y, v, 0.03, 60.0, 82)
    x0 = positive((16, 14), 83)
    x, tr, _ = oracle.run_t(y, v, psf, x0, 60, nu, sr, trace=True)
    assert (np.diff(tr) >= -1e-12 * np.abs(tr[1:])).all()
    assert (x >= 0).all()


def test_scaling_invariance():
    """Scaling y and x0 by s and v by s^2 leaves u (y - Fx)^2 and hence the
    weights unchanged, so the iterates scale by s."""
    y, v, psf, _ = small_problem(10, 9, 3, 3, seed=84, mask=0.1)
    x0 = positive((10, 9), 85)
    a = oracle.run_t(y, v, psf, x0, 5, 3.0)
    b = oracle.run_t(y * np.float32(4), v * np.float32(16), psf, x0 * np.float32(4), 5, 3.0)
    np.testing.assert_allclose(b, 4 * a, rtol=1e-12, atol=1e-12 * np.abs(a).max())


def test_outliers_are_down_weighted():
    """A huge unmasked outlier has a vanishing effect (its weight falls like
    1/residual^2), while Eq. (2) follows it."""
    n, H, W = 4, 8, 8
    y, v, psf, _ = small_problem(H, W, n, 3, seed=86)
    x0 = positive((H, W), 87)
    yo = y.copy()
    yo[2, 4, 4] = np.float32(1e9)
    vm = v.copy()
    vm[2, 4, 4] = np.inf                                 # the same pixel masked
    t_out = oracle.run_t(yo, v, psf, x0, 3, 3.0)
    t_mask = oracle.run_t(y, vm, psf, x0, 3, 3.0)
    g_out = oracle.run(yo, v, psf, x0, 3)
    g_mask = oracle.run(y, vm, psf, x0, 3)
    d_t = np.abs(t_out - t_mask).max() / np.abs(t_mask).max()
    d_g = np.abs(g_out - g_mask).max() / np.abs(g_mask).max()
    assert d_t < 1e-5 and d_g > 1.0


@pytest.mark.parametrize("sr", [1, 2])
def test_step_at_matches_one_step(sr):
    """The pointwise step (used at full size) equals a whole Student-t step."""
    y, v, psf, _ = small_problem(14, 12, 3, 5, sr=sr, seed=90 + sr, mask=0.1)
    y, _ = with_outliers(y, v, 0.05, 30.0, 92)
    x0 = positive((14, 12), 93)
    B, D = oracle.terms_t(y, v, psf, x0, 2.0, sr)
    x1 = oracle.run_t(y, v, psf, x0, 1, 2.0, sr)
    rows = np.array([0, 13, 7, 3, 0], np.int32)
    cols = np.array([0, 11, 5, 9, 11], np.int32)
    Bs, Ds, xs = oracle.step_at(y, v, psf, x0, rows, cols, sr, nu=2.0)
    np.testing.assert_allclose(Bs, B[rows, cols], rtol=1e-12, atol=1e-12 * np.abs(B).max())
    np.testing.assert_allclose(Ds, D[rows, cols], rtol=1e-12)
    np.testing.assert_allclose(xs, x1[rows, cols], rtol=1e-12)


def test_rejects_bad_nu():
    y, v, psf, _ = small_problem(6, 6, 2, 3, seed=88)
    with pytest.raises(ValueError):
        oracle.run_t(y, v, psf, positive((6, 6), 89), 2, 0.0)
