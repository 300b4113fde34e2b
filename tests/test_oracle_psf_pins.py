"""Pins of the oracle's Eq. (4) (super-resolved PSFs by projected Adam).

The objective is checked against a construction from library routines
(scipy.signal.convolve2d, numpy differences); its gradient against exact
central differences (the objective is quadratic); the fit against closed
forms (no blur and no down-sampling: a DST-I solve; lambda = 0: h = f), against
the exact non-negative least-squares minimiser found by enumerating active sets
on a tiny stamp, against the closed form of the first Adam step, and against
exact scale equivariance.  A dropped term, a wrong sign, a wrong index, an
off-by-one anchor or a transposed operand in the oracle breaks one of them.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.fft
import scipy.optimize
import scipy.signal

import oracle
from paper_2302_05804_amd import synth

RNG = np.random.default_rng


# ---------------------------------------------------------------------------
# helpers written from the definitions (not from the oracle)
# ---------------------------------------------------------------------------

def gauss(sigma):
    if sigma == 0:
        return np.ones((1, 1))
    r = math.ceil(4 * sigma)
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(t[:, None] ** 2 + t[None, :] ** 2) / (2 * sigma ** 2))
    return g / g.sum()


def model_lib(h, kf, D, sigma):
    """D(h * g) on f's stamp: full convolution placed with h's centre on fine
    pixel D*(kf-1)/2, clipped to the D*kf stamp, then D x D block sums."""
    g = gauss(sigma)
    hg = scipy.signal.convolve2d(h, g, mode="full")
    c = (h.shape[0] - 1) // 2 + (g.shape[0] - 1) // 2     # centre of hg
    S, a = D * kf, D * ((kf - 1) // 2)
    fine = np.zeros((S + 2 * hg.shape[0], S + 2 * hg.shape[0]))
    off = hg.shape[0]                                      # margin so slicing never clips
    fine[off + a - c:off + a - c + hg.shape[0], off + a - c:off + a - c + hg.shape[1]] = hg
    fine = fine[off:off + S, off:off + S]
    return fine.reshape(kf, D, kf, D).sum(axis=(1, 3))


def penalty_lib(h):
    hp = np.pad(h, 1)
    return (np.diff(hp, axis=0) ** 2).sum() + (np.diff(hp, axis=1) ** 2).sum()


def objective_lib(f, h, D, sigma, lam):
    return ((model_lib(h, f.shape[0], D, sigma) - f) ** 2).sum() + lam * penalty_lib(h)


def dense_problem(kf, kh, D, sigma, lam):
    """(M, rows of sqrt(lam) * differences): objective = |M h - f|^2 + |G h|^2."""
    n = kh * kh
    M = np.stack([model_lib(np.eye(n)[i].reshape(kh, kh), kf, D, sigma).ravel()
                  for i in range(n)], axis=1)
    rows = []
    for i in range(-1, kh):
        for j in range(kh):
            r = np.zeros((kh + 2, kh + 2))
            r[i + 1, j + 1] -= 1
            r[i + 2, j + 1] += 1
            rows.append(r[1:-1, 1:-1].ravel())
    for i in range(kh):
        for j in range(-1, kh):
            r = np.zeros((kh + 2, kh + 2))
            r[i + 1, j + 1] -= 1
            r[i + 1, j + 2] += 1
            rows.append(r[1:-1, 1:-1].ravel())
    return M, math.sqrt(lam) * np.array(rows)


def psf(kf, seed, dy=0.0, dx=0.0):
    rng = RNG(seed)
    return synth.moffat_psf(kf, rng.uniform(2.5, 4.0), rng.uniform(2.5, 4.5), rng.uniform(0, 0.3),
                            rng.uniform(0, math.pi), dy, dx).astype(np.float32)


# ---------------------------------------------------------------------------
# g, objective, gradient, start
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("sigma", [0.0, 0.7, 1.0, 2.0, 3.3])
def test_gauss_definition(sigma):
    g = oracle.psf_gauss(sigma)
    r = math.ceil(4 * sigma)
    assert g.shape == (2 * r + 1, 2 * r + 1)
    assert abs(g.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(g, g.T, rtol=0, atol=1e-18)
    np.testing.assert_allclose(g, g[::-1, ::-1], rtol=0, atol=1e-18)
    if sigma > 0:
        assert abs(g[r, r + 1] / g[r, r] - math.exp(-1 / (2 * sigma ** 2))) < 1e-14
        s = np.linalg.svd(g, compute_uv=False)                     # isotropic Gaussian: rank 1
        assert s[1] < 1e-14 * s[0]


@pytest.mark.parametrize("kf,kh,D,sigma", [(15, 15, 2, 2.0), (9, 21, 2, 1.3), (7, 7, 1, 0.0),
                                           (5, 19, 3, 3.0), (11, 13, 4, 0.7), (3, 9, 2, 1.0)])
def test_objective_matches_library_construction(kf, kh, D, sigma):
    """Includes h wider than the fine stamp (kh > D kf): the clipped part is not seen."""
    rng = RNG(kf * 100 + kh)
    f = psf(kf, kh)
    h = rng.uniform(0, 0.01, (kh, kh))
    J, m = oracle.psf_objective(f, h, D, sigma, 0.03)
    np.testing.assert_allclose(m, model_lib(h, kf, D, sigma), rtol=1e-12, atol=1e-18)
    ref = objective_lib(f.astype(np.float64), h, D, sigma, 0.03)
    assert abs(J - ref) <= 1e-12 * ref


def test_model_anchor_and_phase():
    """A unit impulse at h's centre with no blur lands, through D, on f's centre
    pixel; moving it by one fine pixel down-right stays in that coarse pixel
    (the block of coarse pixel I is fine rows D*I .. D*I+D-1)."""
    kf, kh, D = 5, 7, 2
    h = np.zeros((kh, kh))
    h[3, 3] = 1.0
    _, m = oracle.psf_objective(np.zeros((kf, kf), np.float32), h, D, 0.0, 0.0)
    e = np.zeros((kf, kf))
    e[2, 2] = 1.0
    np.testing.assert_array_equal(m, e)
    h = np.zeros((kh, kh))
    h[4, 4] = 1.0
    _, m = oracle.psf_objective(np.zeros((kf, kf), np.float32), h, D, 0.0, 0.0)
    np.testing.assert_array_equal(m, e)
    h = np.zeros((kh, kh))
    h[2, 3] = 1.0
    _, m = oracle.psf_objective(np.zeros((kf, kf), np.float32), h, D, 0.0, 0.0)
    e = np.zeros((kf, kf))
    e[1, 2] = 1.0
    np.testing.assert_array_equal(m, e)


@pytest.mark.parametrize("kf,kh,D,sigma,lam", [(9, 11, 2, 2.0, 0.02), (5, 9, 3, 1.0, 0.5),
                                               (7, 7, 1, 0.0, 1.0)])
def test_gradient_is_exact_derivative(kf, kh, D, sigma, lam):
    """The objective is quadratic, so central differences are exact up to rounding."""
    rng = RNG(7 + kh)
    f = psf(kf, 3)
    h = rng.uniform(0, 0.02, (kh, kh))
    g = oracle.psf_gradient(f, h, D, sigma, lam)
    for k in range(6):
        e = rng.normal(size=(kh, kh))
        t = 1e-3
        jp, _ = oracle.psf_objective(f, h + t * e, D, sigma, lam)
        jm, _ = oracle.psf_objective(f, h - t * e, D, sigma, lam)
        fd = (jp - jm) / (2 * t)
        assert abs(fd - (g * e).sum()) <= 1e-9 * (abs(fd) + np.abs(g).sum() * np.abs(e).max())
    # pixel by pixel on a corner and the centre (a transposed index fails here)
    for (a, b) in [(0, 0), (0, kh - 1), (kh // 2, kh // 2), (kh - 1, 1)]:
        e = np.zeros((kh, kh))
        e[a, b] = 1.0
        jp, _ = oracle.psf_objective(f, h + 1e-3 * e, D, sigma, lam)
        jm, _ = oracle.psf_objective(f, h - 1e-3 * e, D, sigma, lam)
        assert abs((jp - jm) / 2e-3 - g[a, b]) <= 1e-8 * np.abs(g).max()


@pytest.mark.parametrize("kf,kh,D", [(15, 43, 2), (9, 9, 3), (5, 31, 2), (7, 7, 1)])
def test_start_is_flux_sharing_replication(kf, kh, D):
    f = psf(kf, 5)
    f[0, 0] = -0.01                                   # negative values start at 0
    fine = np.repeat(np.repeat(np.maximum(f.astype(np.float64), 0), D, 0), D, 1) / D ** 2
    a, c = D * ((kf - 1) // 2), (kh - 1) // 2
    pad = kh
    big = np.zeros((fine.shape[0] + 2 * pad, fine.shape[1] + 2 * pad))
    big[pad:-pad, pad:-pad] = fine
    ref = big[pad + a - c:pad + a + c + 1, pad + a - c:pad + a + c + 1]
    np.testing.assert_array_equal(oracle.psf_start(f, kh, D), ref)


# ---------------------------------------------------------------------------
# the fit
# ---------------------------------------------------------------------------

def test_fit_no_blur_no_downsampling_is_dst_solve():
    """D = 1, g = impulse, Kh = Kf: the minimiser of |h - f|^2 + lam |grad h|^2
    is (I + lam L)^-1 f with L the zero-boundary Laplacian, diagonal in the
    DST-I basis.  (I + lam L) is an M-matrix, so f >= 0 gives h >= 0 and the
    constraint is inactive."""
    kf, lam = 15, 0.5
    f = psf(kf, 11)
    k = np.arange(1, kf + 1)
    ev = 4 * np.sin(np.pi * k / (2 * (kf + 1))) ** 2
    den = 1 + lam * (ev[:, None] + ev[None, :])
    exact = scipy.fft.idstn(scipy.fft.dstn(f.astype(np.float64), type=1) / den, type=1)
    assert exact.min() > 0
    h, obj = oracle.psf_fit(f, kf, 1, sigma=0.0, lam=lam, steps=3000)
    assert np.linalg.norm(h[0] - exact) <= 1e-6 * np.linalg.norm(exact)
    h0, _ = oracle.psf_fit(f, kf, 1, sigma=0.0, lam=0.0, steps=3000)
    assert np.abs(h0[0] - f).max() <= 1e-6 * f.max()


def test_fit_reaches_enumerated_nnls_minimiser():
    """Tiny stamp (3 x 3 fine, 9 unknowns), f with negative values so that the
    constraint binds: the exact minimiser over h >= 0 is found by solving the
    normal equations on every one of the 2^9 free sets and keeping the one that
    satisfies the optimality conditions; scipy's NNLS agrees; Adam reaches it."""
    kf, kh, D, sigma, lam = 3, 3, 2, 0.8, 0.05
    f = np.array([[0.02, 0.10, -0.25], [0.15, 0.40, -0.25], [-0.28, -0.22, 0.30]], np.float32)
    M, G = dense_problem(kf, kh, D, sigma, lam)
    A = np.vstack([M, G])
    b = np.concatenate([f.astype(np.float64).ravel(), np.zeros(G.shape[0])])
    Q, q = A.T @ A, A.T @ b
    best = None
    for free in itertools.product([0, 1], repeat=kh * kh):
        F = np.array(free, bool)
        x = np.zeros(kh * kh)
        if F.any():
            x[F] = np.linalg.solve(Q[np.ix_(F, F)], q[F])
        grad = Q @ x - q
        if (x >= -1e-14).all() and (np.abs(grad[F]) < 1e-12).all() and (grad[~F] >= -1e-12).all():
            assert best is None or np.allclose(best, x, atol=1e-12)     # unique minimiser
            best = x
    assert best is not None and 2 <= (best == 0).sum() <= 6
    nn, _ = scipy.optimize.nnls(A, b)
    np.testing.assert_allclose(nn, best, atol=1e-10)
    h, obj = oracle.psf_fit(f, kh, D, sigma=sigma, lam=lam, steps=4000)
    assert np.abs(h[0].ravel() - best).max() <= 1e-6 * np.abs(best).max()
    assert abs(obj[0] - ((A @ best - b) ** 2).sum()) <= 1e-9


def test_fit_first_step_closed_form():
    """After one step Adam's bias-corrected ratio is g / (|g| + eps):
    h1 = max(0, h0 - lr max(f) g / (|g| + eps)) with g the gradient at the start."""
    f = psf(11, 13)
    kh, D, lr, eps = 15, 2, 0.05, 1e-7
    h0 = oracle.psf_start(f, kh, D)
    g = oracle.psf_gradient(f, h0, D, 2.0, 0.01)
    ref = np.maximum(0.0, h0 - lr * float(f.max()) * g / (np.abs(g) + eps))
    h1, _ = oracle.psf_fit(f, kh, D, lam=0.01, steps=1, lr=lr, eps=eps)
    np.testing.assert_allclose(h1[0], ref, rtol=1e-14, atol=1e-20)
    # an explicit start is used as given
    hs = RNG(1).uniform(0, 0.01, (1, kh, kh)).astype(np.float32)
    hz, _ = oracle.psf_fit(f, kh, D, h0=hs, steps=0)
    np.testing.assert_array_equal(hz[0], hs[0].astype(np.float64))


def test_fit_scale_equivariance():
    """Scaling f (and Adam's eps) by 2^k scales every iterate by 2^k exactly:
    the gradient is linear in (h, f), the step is relative to max(f)."""
    f = psf(13, 17)
    a, _ = oracle.psf_fit(f, 17, 2, steps=300)
    b, _ = oracle.psf_fit(f * np.float32(8.0), 17, 2, steps=300, eps=8e-7)
    np.testing.assert_array_equal(b, 8.0 * a)


def test_fit_optimality_and_descent():
    """A realistic stamp (Kf = 15, Kh = 21, Delta = 2, sigma = 2): the result
    satisfies the optimality conditions of Eq. (4) to a small fraction of the
    initial gradient, and the objective fell from the start."""
    f = psf(15, 19, 0.3, 0.6)
    h, obj = oracle.psf_fit(f, 21, 2, steps=3000)
    j0, _ = oracle.psf_objective(f, oracle.psf_start(f, 21, 2), 2, 2.0, 1e-2)
    assert obj[0] < 0.5 * j0
    g0 = np.abs(oracle.psf_gradient(f, oracle.psf_start(f, 21, 2), 2, 2.0, 1e-2)).max()
    g = oracle.psf_gradient(f, h[0], 2, 2.0, 1e-2)
    pos = h[0] > 0
    assert np.abs(g[pos]).max() <= 1e-3 * g0
    assert (g[~pos] >= -1e-3 * g0).all()
    assert (h >= 0).all()


def test_fit_rejects_bad_arguments():
    f = psf(9, 1)
    with pytest.raises(ValueError):
        oracle.psf_fit(f, 10, 2)
    with pytest.raises(ValueError):
        oracle.psf_fit(f, 9, 5)
    with pytest.raises(ValueError):
        oracle.psf_gauss(9.0)


def test_fit_second_step_closed_form():
    """Two steps (S = 2): the second uses the decayed step lr max(f) decay and
    Adam's bias-corrected moments of the two gradients (Kingma & Ba, Alg. 1)."""
    f = psf(11, 23)
    kh, D, lr, dec, b1, b2, eps = 13, 2, 0.03, 0.1, 0.9, 0.999, 1e-7
    h0 = oracle.psf_start(f, kh, D)
    g1 = oracle.psf_gradient(f, h0, D, 2.0, 0.01)
    h1 = np.maximum(0.0, h0 - lr * float(f.max()) * g1 / (np.abs(g1) + eps))
    g2 = oracle.psf_gradient(f, h1, D, 2.0, 0.01)
    m = b1 * (1 - b1) * g1 + (1 - b1) * g2
    v = b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2
    step = lr * float(f.max()) * dec * (m / (1 - b1 ** 2)) / (np.sqrt(v / (1 - b2 ** 2)) + eps)
    ref = np.maximum(0.0, h1 - step)
    h2, _ = oracle.psf_fit(f, kh, D, lam=0.01, steps=2, lr=lr, decay=dec)
    np.testing.assert_allclose(h2[0], ref, rtol=1e-12, atol=1e-18)
