"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same
seeded inputs and compare."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_run(y, v, psf, sr, n_iter, x0=None, precision=0, trace=True):
    """Run n_iter EM iterations through the C ABI; returns (x, trace)."""
    import torch
    from paper_2302_05804_amd import em
    n, hf, wf = y.shape
    p = em.Problem.make(n, hf, wf, psf.shape[1], sr=sr, precision=precision)
    yd, vd, fd = to_dev(y), to_dev(v), to_dev(psf)
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    x0d = to_dev(x0) if x0 is not None else None
    ctx = em.Context(p, yd, vd, fd, x, x0=x0d)
    tr = ctx.iterate(n_iter, trace=trace)
    ctx.sync()
    out = x.cpu().numpy().astype(np.float64)
    ctx.close()
    return out, tr
