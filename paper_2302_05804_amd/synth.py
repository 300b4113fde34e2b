"""Seeded synthetic inputs shaped like the paper's workloads.

The paper's Hyper Suprime-Cam exposures (33 frames of 4K x 4K, 43 x 43 PSFs;
Sec. 2, Fig. 1) are not available, so these generators stand in for them with
the same shapes and with value distributions chosen from what the paper says
about the data (sky-subtracted exposures with Gaussian noise of per-pixel
variance, Eq. (1); per-exposure PSFs; variance maps; artefacts such as
cosmic-ray streaks and bad columns marked as masked pixels).

This module only *synthesises* data.  It holds none of the EM method's
arithmetic (no weighting, no adjoint, no update); the one convolution it needs
to render the exposures is done with scipy's FFT.  Both the oracle (``oracle/``)
and the GPU path receive its arrays; neither imports the other.

Conventions shared with the method's definition (so the model is exact at the
edges): PSFs are K x K with odd K, centred at c = (K-1)/2; "same"-size
zero-filled convolution; a 2 x 2 box *sum* from the latent grid to the frame grid
when the super-resolution factor is 2.  Masked pixels carry v = +inf and
y = NaN.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.fft as sfft

# ----------------------------------------------------------------------------
# PSF models
# ----------------------------------------------------------------------------


def _ellipse_r2(K: int, scale_major: float, q: float, theta: float, dy: float, dx: float):
    """Elliptical squared radius on a K x K stamp centred at (c+dy, c+dx).

    Axis ratio q = b/a, the geometric-mean scale is kept: a = s/sqrt(q), b = s*sqrt(q).
    """
    c = (K - 1) / 2.0
    yy, xx = np.mgrid[0:K, 0:K].astype(np.float64)
    yy -= c + dy
    xx -= c + dx
    ct, st = math.cos(theta), math.sin(theta)
    u = ct * xx + st * yy
    w = -st * xx + ct * yy
    a = scale_major / math.sqrt(q)
    b = scale_major * math.sqrt(q)
    return (u / a) ** 2 + (w / b) ** 2


def gaussian_psf(K: int, fwhm: float, ellipticity: float, theta: float,
                 dy: float = 0.0, dx: float = 0.0) -> np.ndarray:
    """Elliptical Gaussian, geometric-mean sigma = FWHM / 2.3548, normalised to 1."""
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    r2 = _ellipse_r2(K, sigma, 1.0 - ellipticity, theta, dy, dx)
    p = np.exp(-0.5 * r2)
    return p / p.sum()


def moffat_psf(K: int, fwhm: float, beta: float, ellipticity: float, theta: float,
               dy: float = 0.0, dx: float = 0.0) -> np.ndarray:
    """Elliptical Moffat (1 + (r/alpha)^2)^-beta, alpha = FWHM / (2 sqrt(2^(1/beta) - 1))."""
    alpha = fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))
    r2 = _ellipse_r2(K, alpha, 1.0 - ellipticity, theta, dy, dx)
    p = (1.0 + r2) ** (-beta)
    return p / p.sum()


# ----------------------------------------------------------------------------
# Sky model: point sources + Sersic galaxies on a zero background
# ----------------------------------------------------------------------------


def sersic_bn(n: float) -> float:
    """Ciotti & Bertin (1999) asymptotic expansion of b_n."""
    return (2.0 * n - 1.0 / 3.0 + 4.0 / (405.0 * n) + 46.0 / (25515.0 * n * n)
            + 131.0 / (1148175.0 * n ** 3))


def render_sky(H: int, W: int, n_points: int, n_gal: int, rng: np.random.Generator,
               point_flux=(1e2, 1e5), gal_flux=(1e3, 1e5), re_range=(3.0, 8.0),
               n_range=(1.0, 4.0), scale: float = 1.0) -> np.ndarray:
    """Latent sky x >= 0: single-pixel point sources (flux log-uniform) and
    Sersic galaxies I ~ exp(-b_n [(r/r_e)^(1/n) - 1]) with total flux log-uniform.
    ``scale`` multiplies galaxy radii (latent pixels per frame pixel for SR)."""
    x = np.zeros((H, W), np.float64)
    if n_points:
        py = rng.integers(0, H, n_points)
        px = rng.integers(0, W, n_points)
        fl = np.exp(rng.uniform(math.log(point_flux[0]), math.log(point_flux[1]), n_points))
        np.add.at(x, (py, px), fl)
    for _ in range(n_gal):
        n = rng.uniform(*n_range)
        re = rng.uniform(*re_range) * scale
        q = rng.uniform(0.4, 1.0)
        th = rng.uniform(0.0, math.pi)
        flux = math.exp(rng.uniform(math.log(gal_flux[0]), math.log(gal_flux[1])))
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        R = int(min(max(6.0 * re, 8.0), 64.0 * scale))
        y0, y1 = max(int(cy) - R, 0), min(int(cy) + R + 1, H)
        x0, x1 = max(int(cx) - R, 0), min(int(cx) + R + 1, W)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
        yy += 0.5 - cy
        xx += 0.5 - cx
        ct, st = math.cos(th), math.sin(th)
        u = ct * xx + st * yy
        w = -st * xx + ct * yy
        r = np.sqrt(u * u / q + w * w * q)
        prof = np.exp(-sersic_bn(n) * ((r / re) ** (1.0 / n) - 1.0))
        s = prof.sum()
        if s > 0:
            x[y0:y1, x0:x1] += flux * prof / s
    return x


# ----------------------------------------------------------------------------
# Rendering exposures (data synthesis; scipy FFT)
# ----------------------------------------------------------------------------


class _SameConv:
    """'same'-size zero-filled convolution of one latent image with many PSFs."""

    def __init__(self, x: np.ndarray, K: int):
        self.H, self.W = x.shape
        self.K = K
        self.s = (sfft.next_fast_len(self.H + K - 1, real=True),
                  sfft.next_fast_len(self.W + K - 1, real=True))
        self.X = sfft.rfft2(x, self.s, workers=-1)

    def __call__(self, f: np.ndarray) -> np.ndarray:
        c = (self.K - 1) // 2
        F = sfft.rfft2(f, self.s, workers=-1)
        full = sfft.irfft2(self.X * F, self.s, workers=-1)
        return full[c:c + self.H, c:c + self.W]


def _box2(z: np.ndarray) -> np.ndarray:
    H, W = z.shape
    return z.reshape(H // 2, 2, W // 2, 2).sum(axis=(1, 3))


def _streak_mask(H: int, W: int, frac: float, rng: np.random.Generator) -> np.ndarray:
    """Cosmic-ray streaks (1-2 px wide, 5-50 px long, random angle) and bad
    columns (full or partial), together covering about ``frac`` of the pixels."""
    m = np.zeros((H, W), bool)
    target = frac * H * W
    # bad columns: about 30% of the masked area
    col_budget = 0.3 * target
    while col_budget > 0:
        col = rng.integers(0, W)
        if rng.uniform() < 0.5:
            r0, r1 = 0, H
        else:
            r0 = int(rng.integers(0, H))
            r1 = min(H, r0 + int(rng.integers(H // 8 + 1, H // 2 + 2)))
        m[r0:r1, col] = True
        col_budget -= (r1 - r0)
    # streaks for the rest
    n_streak = max(1, int(0.7 * target / 41.0))
    L = rng.uniform(5, 50, n_streak)
    wdt = rng.integers(1, 3, n_streak)
    ang = rng.uniform(0, math.pi, n_streak)
    cy = rng.uniform(0, H, n_streak)
    cx = rng.uniform(0, W, n_streak)
    steps = np.arange(0, 50.5, 0.5)
    for k in range(n_streak):
        s = steps[steps <= L[k]] - L[k] / 2
        yy = cy[k] + s * math.sin(ang[k])
        xx = cx[k] + s * math.cos(ang[k])
        for d in range(int(wdt[k])):
            iy = np.clip((yy + d * math.cos(ang[k])).astype(np.int64), 0, H - 1)
            ix = np.clip((xx - d * math.sin(ang[k])).astype(np.int64), 0, W - 1)
            m[iy, ix] = True
    return m


@dataclasses.dataclass
class Problem:
    """One synthetic multi-frame problem (all arrays C-contiguous)."""
    name: str
    y: np.ndarray          # n x Hf x Wf float32 exposures (NaN where masked)
    v: np.ndarray          # n x Hf x Wf float32 variances (+inf where masked)
    psf: np.ndarray        # n x K x K float32 PSFs on the latent grid
    x_true: np.ndarray     # Hl x Wl float64 latent sky used to render y
    sr: int                # super-resolution factor (1 or 2)
    n_iter: int            # iterations the workload runs
    seed: int

    @property
    def n(self) -> int:
        return self.y.shape[0]

    @property
    def frame_shape(self):
        return self.y.shape[1:]

    @property
    def latent_shape(self):
        return (self.y.shape[1] * self.sr, self.y.shape[2] * self.sr)

    @property
    def K(self) -> int:
        return self.psf.shape[1]


# Recipes of the five workloads (latent size, frames, PSF, sky, noise, masks).
CONFIGS = {
    # oracle-size plain EM
    "c1": dict(H=128, W=128, n=4, K=15, sr=1, psf="gauss", fwhm=(2.0, 4.0), ell=0.2,
               points=20, gals=3, sky=(10.0, 10.0), mask=0.0, mask_kind="none", n_iter=30),
    # plain FP32 GPU size
    "c2": dict(H=1024, W=1024, n=8, K=43, sr=1, psf="moffat", fwhm=(3.0, 6.0), ell=0.3,
               points=2000, gals=200, sky=(50.0, 200.0), mask=0.02, mask_kind="pixels",
               n_iter=100),
    # HSC-shaped batch
    "c3": dict(H=4096, W=4096, n=33, K=43, sr=1, psf="moffat", fwhm=(3.0, 7.0), ell=0.3,
               points=32000, gals=3200, sky=(50.0, 500.0), mask=0.01, mask_kind="streaks",
               n_iter=100),
    # super-resolution x2 (H, W are the latent size; frames are half of it)
    "c4": dict(H=4096, W=4096, n=16, K=43, sr=2, psf="moffat", fwhm=(3.0, 6.0), ell=0.3,
               points=32000, gals=3200, sky=(50.0, 200.0), mask=0.02, mask_kind="pixels",
               n_iter=100),
}
CONFIG_INDEX = {"c1": 1, "c2": 2, "c3": 3, "c4": 4, "c5": 5}


def make_problem(config: str = "c1", replica: int = 0, seed: Optional[int] = None,
                 **over) -> Problem:
    """Build a seeded problem following recipe ``config`` ('c1'..'c4').

    Keyword overrides (H, W = latent size, n, K, n_iter, points, gals, mask ...)
    rescale the recipe; source counts scale with the latent area unless given.
    Seed = 1000 * config index + replica unless given explicitly.
    """
    rec = dict(CONFIGS[config])
    base_area = rec["H"] * rec["W"]
    rec.update(over)
    if ("H" in over or "W" in over) and "points" not in over:
        rec["points"] = max(1, int(round(CONFIGS[config]["points"] * rec["H"] * rec["W"] / base_area)))
    if ("H" in over or "W" in over) and "gals" not in over:
        rec["gals"] = int(round(CONFIGS[config]["gals"] * rec["H"] * rec["W"] / base_area))
    if seed is None:
        seed = 1000 * CONFIG_INDEX[config] + replica
    rng = np.random.Generator(np.random.PCG64(seed))
    H, W, n, K, sr = rec["H"], rec["W"], rec["n"], rec["K"], rec["sr"]
    if H % sr or W % sr:
        raise ValueError("latent size must be a multiple of sr")
    if K % 2 == 0:
        raise ValueError("K must be odd")
    Hf, Wf = H // sr, W // sr

    x = render_sky(H, W, rec["points"], rec["gals"], rng, scale=float(sr))
    conv = _SameConv(x, K)

    psfs = np.empty((n, K, K), np.float32)
    y = np.empty((n, Hf, Wf), np.float32)
    v = np.empty((n, Hf, Wf), np.float32)
    for t in range(n):
        fwhm = rng.uniform(*rec["fwhm"]) * sr       # PSF width in latent pixels
        e = rng.uniform(0.0, rec["ell"])
        th = rng.uniform(0.0, math.pi)
        dy, dx = (rng.uniform(0.0, 1.0, 2) if sr == 2 else (0.0, 0.0))
        if rec["psf"] == "gauss":
            p = gaussian_psf(K, fwhm, e, th, dy, dx)
        else:
            beta = rng.uniform(2.5, 4.5)
            p = moffat_psf(K, fwhm, beta, e, th, dy, dx)
        psfs[t] = p.astype(np.float32)
        model = conv(psfs[t].astype(np.float64))
        if sr == 2:
            model = _box2(model)
        model = np.maximum(model, 0.0)
        s_t = rng.uniform(*rec["sky"])
        var = s_t + model
        noise = rng.standard_normal((Hf, Wf), dtype=np.float32).astype(np.float64)
        y[t] = (model + np.sqrt(var) * noise).astype(np.float32)
        v[t] = var.astype(np.float32)
        if rec["mask"] > 0:
            if rec["mask_kind"] == "pixels":
                mk = rng.uniform(size=(Hf, Wf)) < rec["mask"]
            else:
                mk = _streak_mask(Hf, Wf, rec["mask"], rng)
            y[t][mk] = np.nan
            v[t][mk] = np.inf
    return Problem(name=config, y=y, v=v, psf=psfs, x_true=x, sr=sr,
                   n_iter=int(rec["n_iter"]), seed=int(seed))


def add_trails(y: np.ndarray, v: np.ndarray, seed: int, per_frame=(1, 2), width=(2, 4),
               amp=(20.0, 200.0)):
    """Unflagged satellite trails (outliers the variance map does not know
    about): per frame U{per_frame} straight lines across the whole frame, width
    U{width} px, adding amp ~ U(amp) standard deviations sqrt(v) on the line
    (masked pixels untouched).  Returns (new y, boolean trail mask)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y = y.copy()
    n, H, W = y.shape
    hit = np.zeros(y.shape, bool)
    L = math.hypot(H, W)
    steps = np.arange(-L / 2, L / 2, 0.5)
    for t in range(n):
        for _ in range(int(rng.integers(per_frame[0], per_frame[1] + 1))):
            ang = rng.uniform(0, math.pi)
            cy, cx = rng.uniform(0, H), rng.uniform(0, W)
            wd = int(rng.integers(width[0], width[1] + 1))
            for d in range(wd):
                yy = cy + steps * math.sin(ang) + d * math.cos(ang)
                xx = cx + steps * math.cos(ang) - d * math.sin(ang)
                ok = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W)
                hit[t, yy[ok].astype(np.int64), xx[ok].astype(np.int64)] = True
        a = rng.uniform(*amp)
        m = hit[t] & np.isfinite(v[t])
        y[t][m] += (a * np.sqrt(v[t][m].astype(np.float64))).astype(np.float32)
    return y, hit


def coarse_psfs(n: int, kf: int = 43, factor: int = 2, seed: int = 4100,
                fwhm=(3.0, 6.0), ell: float = 0.3) -> np.ndarray:
    """n frame-grid PSFs (kf x kf, float32) to be super-resolved by Eq. (4):
    elliptical Moffat, FWHM ~ U(fwhm) frame pixels, beta ~ U(2.5, 4.5),
    ellipticity ~ U(0, ell), random angle, centre offset ~ U[0, 1)^2 fine
    pixels (U[0, 1/factor)^2 frame pixels), unit sum."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, kf, kf), np.float32)
    for t in range(n):
        fw = rng.uniform(*fwhm)
        beta = rng.uniform(2.5, 4.5)
        e = rng.uniform(0.0, ell)
        th = rng.uniform(0.0, math.pi)
        dy, dx = rng.uniform(0.0, 1.0, 2) / factor
        out[t] = moffat_psf(kf, fw, beta, e, th, dy, dx).astype(np.float32)
    return out


def positive_start(shape, level: float, seed: int, spread: float = 0.5) -> np.ndarray:
    """A strictly positive, non-flat starting guess: level * U(1-spread, 1+spread)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (level * rng.uniform(1.0 - spread, 1.0 + spread, size=shape)).astype(np.float32)


# ----------------------------------------------------------------------------
# Serving stream (workload 5): job descriptions with Poisson arrivals
# ----------------------------------------------------------------------------


@dataclasses.dataclass
class JobSpec:
    frame_side: int
    n: int
    sr: int
    n_iter: int
    arrival: float
    seed: int


def serving_stream(n_jobs: int, rate: float, seed: int = 5000, side=(256, 2048),
                   frames=(4, 33), iters=(50, 200)):
    """Jobs with frame side log-uniform in ``side`` (multiple of 64), n uniform in
    ``frames``, sr in {1, 2}, iterations uniform in ``iters``, Poisson arrivals."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate)
        s = math.exp(rng.uniform(math.log(side[0]), math.log(side[1])))
        s = max(64, int(round(s / 64.0)) * 64)
        out.append(JobSpec(frame_side=s, n=int(rng.integers(frames[0], frames[1] + 1)),
                           sr=int(rng.integers(1, 3)),
                           n_iter=int(rng.integers(iters[0], iters[1] + 1)),
                           arrival=t, seed=seed * 10 + j))
    return out
