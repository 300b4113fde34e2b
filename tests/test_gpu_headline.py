"""Parity at the headline configurations' frame and iteration counts.

* c3crop: the HSC-shaped recipe with all 33 frames (43 x 43 Moffat PSFs,
  cosmic-ray streaks and bad columns masked) on a 272 x 200 crop (tiles of 128
  with ragged tails in both directions), 100 iterations of Eq. (2) from the
  flat start, in every precision, in the kernel variants the benchmark's
  autotuner picks on the full 33 x 4096^2 job (FP16 split: forward 2, adjoint
  2; BF16 split: forward 0, adjoint 2) and in the default ones.  Checked
  against the oracle's iterates after 10, 50 and 100 iterations and its
  log-likelihood trace l(x^(k-1)), k = 1..100.
* sr2job: a super-resolution x2 job of the serving stream's kind (Eq. (3); 4
  frames of 72 x 152 on a 144 x 304 latent grid, wider than two 128-column
  tiles and not a multiple of 128), 60 iterations, served in the FP16 split
  form by em_submit and run alone in every adjoint variant.

Expected values: tests/golden/*.npz, written by tests/golden/make_golden.py
from the FP64 oracle alone.  Bars: x rel L2 <= 1e-5 and the trace within 1e-6
relative (FP32); 1e-3 for both in the split forms.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from tests.gpu_common import log, rel_l2, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
if GOLDEN not in sys.path:
    sys.path.insert(0, GOLDEN)
import make_golden  # noqa: E402

BARS = {"FP32": (1e-5, 1e-6), "BF16_SPLIT": (1e-3, 1e-3), "FP16_SPLIT": (1e-3, 1e-3)}


def _golden(case):
    z = np.load(os.path.join(GOLDEN, f"{case}.npz"), allow_pickle=False)
    p, x0 = make_golden.inputs(case)
    assert str(z["digest"]) == make_golden.input_digest(p), "inputs no longer match the golden"
    assert np.array_equal(z["x0"], x0)
    return p, x0, z


@pytest.mark.parametrize("form,variants", [("FP32", None), ("BF16_SPLIT", (0, 2)),
                                           ("FP16_SPLIT", (2, 2)), ("BF16_SPLIT", None),
                                           ("FP16_SPLIT", None)])
def test_c3crop_100_iterations(form, variants):
    import torch
    from paper_2302_05804_amd import em
    p, x0, z = _golden("c3crop")
    n, hf, wf = p.y.shape
    log(f"c3crop {form} variants={variants}: frames {p.y.shape}")
    prob = em.Problem.make(n, hf, wf, p.K, precision=getattr(em, form))
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0),
                     stream=torch.cuda.Stream())
    if variants is not None:
        ctx.set_variants(*variants)
    xb, lb = BARS[form]
    trace = []
    done = 0
    for k in (10, 50, 100):
        trace.append(ctx.iterate(k - done, trace=True))
        done = k
        xg = x.cpu().numpy().astype(np.float64)
        err = rel_l2(xg, z[f"x{k}"])
        log(f"  x^({k}): rel L2 {err:.3e}")
        assert err <= xb, (k, err)
    ctx.close()
    tr = np.concatenate(trace)
    llerr = float(np.max(np.abs(tr - z["trace"]) / np.abs(z["trace"])))
    log(f"  loglik trace: max rel err {llerr:.3e}")
    assert llerr <= lb
    # the iterate moved far from the start: the check is not a trivial one
    assert rel_l2(z["x100"], x0) > 0.5


def test_sr2job_served_fp16_matches_oracle():
    from paper_2302_05804_amd import em
    p, x0, z = _golden("sr2job")
    n, hf, wf = p.y.shape
    assert np.all(x0 == np.float32(oracle.flat_x0(p.y, p.v, 2)))
    prob = em.Problem.make(n, hf, wf, p.K, sr=2, precision=em.FP16_SPLIT)
    srv = em.Server(1 << 30, max_slots=2)
    jid = srv.submit(prob, p.y, p.v, p.psf, 60)
    xs, ll = srv.wait(jid)
    srv.close()
    err = rel_l2(xs, z["x60"])
    llo = oracle.loglik(p.y, p.v, p.psf, z["x60"], sr=2)
    llerr = abs(ll - llo) / abs(llo)
    log(f"served sr=2 FP16 job {p.y.shape} -> {p.latent_shape}, 60 iterations: "
        f"rel L2 {err:.3e}, final loglik rel err {llerr:.3e}")
    assert err <= 1e-3
    assert llerr <= 1e-3


@pytest.mark.parametrize("adj", [0, 1, 2])
def test_sr2job_every_adjoint_variant(adj):
    import torch
    from paper_2302_05804_amd import em
    p, x0, z = _golden("sr2job")
    n, hf, wf = p.y.shape
    prob = em.Problem.make(n, hf, wf, p.K, sr=2, precision=em.FP16_SPLIT)
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
    ctx.set_variants(adj, adj)
    tr = ctx.iterate(20, trace=True)
    e20 = rel_l2(x.cpu().numpy(), z["x20"])
    tr2 = ctx.iterate(40, trace=True)
    e60 = rel_l2(x.cpu().numpy(), z["x60"])
    ctx.close()
    llerr = float(np.max(np.abs(np.concatenate([tr, tr2]) - z["trace"]) / np.abs(z["trace"])))
    log(f"sr2job FP16 variants ({adj},{adj}): x^(20) {e20:.3e}, x^(60) {e60:.3e}, "
        f"loglik {llerr:.3e}")
    assert e20 <= 1e-3 and e60 <= 1e-3 and llerr <= 1e-3
