"""The largest problem the library accepts: a latent image (and frames) of
32767 x 65535 pixels, just under 2^31, with the widest accepted frame side
(65535 <= 65536), two frames (so frame offsets pass 2^31), 43 x 43 PSFs.
One EM iteration (Eq. (2)) in FP32, BF16 split and FP16 split against the
oracle evaluated at 12 pixels (corners, last row and column, seeded interior
points), error |x1 - x1_oracle| / max(|x1_oracle|, 0.05 x0).  About 100 GB of
HBM and 45 GB of host memory.
"""
import numpy as np
import pytest

import oracle
from paper_2302_05804_amd import synth
from tests.gpu_common import log

pytestmark = pytest.mark.gpu

H, W, N, K = 32767, 65535, 2, 43
BARS = {"FP32": 1e-5, "BF16_SPLIT": 1e-3, "FP16_SPLIT": 1e-3}


@pytest.fixture(scope="module")
def data():
    import torch
    assert H * W < 2 ** 31 and (N - 1) * H * W + H * W > 2 ** 31
    rng = np.random.default_rng(9100)
    log(f"max-size problem: {N} frames of {H} x {W} ({H * W} pixels each), K={K}")
    y = rng.standard_normal((N, H, W), dtype=np.float32)
    y *= np.float32(10.0)
    y += np.float32(100.0)
    v = rng.random((N, H, W), dtype=np.float32)
    v *= np.float32(100.0)
    v += np.float32(50.0)
    v[0, 5, 7] = np.inf                      # a masked pixel in each frame
    v[1, H - 3, W - 2] = np.inf
    psf = np.stack([synth.moffat_psf(K, 4.0 + t, 3.0, 0.2, 0.5 + t) for t in range(N)]).astype(np.float32)
    x0 = rng.random((H, W), dtype=np.float32)
    x0 *= np.float32(100.0)
    x0 += np.float32(50.0)
    rows = np.concatenate([[0, 0, H - 1, H - 1, H - 1, 3], rng.integers(0, H, 6)]).astype(np.int32)
    cols = np.concatenate([[0, W - 1, 0, W - 1, W // 2, W - 1], rng.integers(0, W, 6)]).astype(np.int32)
    _, _, x1o = oracle.step_at(y, v, psf, x0, rows, cols, 1)
    dev = [torch.from_numpy(a).cuda() for a in (y, v, psf, x0)]
    log("  inputs resident on the GPU")
    return dev, rows, cols, x0[rows, cols].astype(np.float64), x1o


@pytest.mark.parametrize("prec_name", ["FP32", "BF16_SPLIT", "FP16_SPLIT"])
def test_largest_problem(prec_name, data):
    import torch
    from paper_2302_05804_amd import em
    (yd, vd, fd, x0d), rows, cols, x0s, x1o = data
    p = em.Problem.make(N, H, W, K, precision=getattr(em, prec_name))
    x = torch.empty((H, W), dtype=torch.float32, device="cuda")
    ctx = em.Context(p, yd, vd, fd, x, x0=x0d)
    ctx.iterate(1)
    ctx.sync()
    ri = torch.from_numpy(rows.astype(np.int64)).cuda()
    ci = torch.from_numpy(cols.astype(np.int64)).cuda()
    xs = x[ri, ci].double().cpu().numpy()
    ctx.close()
    del ctx, x
    torch.cuda.empty_cache()
    err = np.abs(xs - x1o) / np.maximum(np.abs(x1o), 0.05 * x0s)
    log(f"  {prec_name}: max error at {rows.size} pixels {err.max():.2e}")
    assert err.max() <= BARS[prec_name]
