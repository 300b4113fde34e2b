"""em_run_noalloc, the entry point for callers that cannot allocate: one job in
the library's static per-GPU scratch array.  Checked bit for bit against the
workspace entry point (em_init + em_iterate, default kernel variants, eager
launches) on two calls in a row, the second on a smaller problem (the array
keeps the first call's contents), for the FP32 and FP16 split forms, with and
without the log-likelihood trace; problems beyond the array's size are refused
with EM_ENOMEM before any device work."""
import numpy as np
import pytest

from paper_2302_05804_amd import synth
from tests.gpu_common import log, to_dev

pytestmark = pytest.mark.gpu


def _em():
    from paper_2302_05804_amd import em
    return em


def _reference(p, prec, n_iter, x0):
    import torch
    em = _em()
    n, hf, wf = p.y.shape
    prob = em.Problem.make(n, hf, wf, p.K, sr=p.sr, precision=prec)
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x,
                     x0=None if x0 is None else to_dev(x0))
    tr = ctx.iterate(n_iter, trace=True)
    ctx.sync()
    out = x.cpu().numpy()
    ctx.close()
    return out, tr


def _noalloc(p, prec, n_iter, x0):
    import torch
    em = _em()
    n, hf, wf = p.y.shape
    prob = em.Problem.make(n, hf, wf, p.K, sr=p.sr, precision=prec)
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    tr = em.run_noalloc(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, n_iter,
                        x0=None if x0 is None else to_dev(x0), trace=True)
    return x.cpu().numpy(), tr


@pytest.mark.parametrize("prec", [0, 2])
def test_noalloc_matches_workspace_entry_point_twice(prec):
    cases = [  # (recipe, latent H, W, n, sr, iterations, positive start?)
        ("c2", 200, 264, 4, 1, 6, True),     # several tiles, ragged
        ("c4", 96, 80, 2, 2, 4, False),      # smaller, sr = 2, flat start
    ]
    for k, (rec, H, W, n, sr, it, pos) in enumerate(cases):
        p = synth.make_problem(rec, H=H, W=W, n=n, seed=960 + k)
        x0 = synth.positive_start(p.latent_shape, 20.0, seed=961 + k) if pos else None
        log(f"noalloc prec={prec} call {k + 1}: frames {p.y.shape} sr={sr} iters={it}")
        a, ta = _noalloc(p, prec, it, x0)
        b, tb = _reference(p, prec, it, x0)
        assert np.array_equal(a, b), (prec, k)
        assert np.array_equal(ta, tb), (prec, k)


def test_noalloc_refuses_problems_beyond_its_array():
    import torch
    em = _em()
    n, hf, wf = 8, 2048, 2048   # workspace far above 256 MiB
    prob = em.Problem.make(n, hf, wf, 43)
    assert em.workspace_bytes(prob) > em.NOALLOC_SCRATCH_BYTES
    y = torch.zeros((n, hf, wf), dtype=torch.float32, device="cuda")
    f = torch.zeros((n, 43, 43), dtype=torch.float32, device="cuda")
    x = torch.zeros((hf, wf), dtype=torch.float32, device="cuda")
    with pytest.raises(em.EMError) as ei:
        em.run_noalloc(prob, y, y, f, x, 1)
    assert ei.value.code == em.ENOMEM
    assert float(x.abs().max().item()) == 0.0   # nothing ran
