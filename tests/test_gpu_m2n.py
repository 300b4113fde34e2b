"""The super-resolution (sr = 2, Eq. (3)) split-form forward that puts the
frames in the N dimension of the matrix-core products, used for jobs of at least
8 frames (16 frames per workgroup and 16 x 64 frame pixels in the FP16 split
form, 16 x 32 in the BF16 split form; a last group of fewer frames is padded
with zero PSFs).

Error models as for the other kernels of each form.  FP16 split: binary16 image
operand with a power-of-two tile scale (2^-11 relative), the PSF's hi + lo
binary16 parts on rows 11..32 of the 44-row box-extended kernel and the hi part
alone elsewhere (2^-11), FP32 accumulation; the forward is bounded element by
element by 1e-3 * sum |g||x| (the oracle on absolute values).  BF16 split: hi +
lo bf16 parts of both operands, three products (the dropped lo x lo term is
about 2^-16 relative), FP32 accumulation; bound 1e-4 * sum |g||x|, as for the
other BF16 split operators.  Whole runs stay within rel L2 1e-3 of the oracle.
Every variant of a form accumulates each output's products in the same order, so
the variants agree bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_2302_05804_amd import synth
from tests.gpu_common import gpu_run, log, rel_l2, to_dev

pytestmark = pytest.mark.gpu

OP_EPS = {"FP16_SPLIT": 1e-3, "BF16_SPLIT": 1e-4}
X_TOL = 1e-3
PRECS = ["FP16_SPLIT", "BF16_SPLIT"]


def _em():
    from paper_2302_05804_amd import em
    return em


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("K,hf,wf,n", [(43, 75, 130, 16), (43, 33, 70, 8), (15, 40, 200, 20),
                                       (43, 17, 64, 33), (43, 3, 2, 9), (7, 16, 65, 12)])
def test_m2n_forward_elementwise_bound(K, hf, wf, n, prec):
    em = _em()
    log(f"m2n forward {prec} K={K} frame {hf}x{wf} n={n}")
    rng = np.random.default_rng(K * 31 + hf + n)
    psf = rng.uniform(0, 1, (n, K, K)).astype(np.float32)
    psf /= psf.sum(axis=(1, 2), keepdims=True)
    x = rng.gamma(0.5, 200.0, (2 * hf, 2 * wf)).astype(np.float32)
    p = em.Problem.make(n, hf, wf, K, sr=2, precision=getattr(em, prec))
    m = em.forward_op(p, to_dev(psf), to_dev(x)).cpu().numpy()
    worst = 0.0
    for t in range(n):
        mo = oracle.forward(psf[t], x, 2)
        mb = oracle.forward(np.abs(psf[t]), np.abs(x), 2)
        assert (np.abs(m[t] - mo) <= OP_EPS[prec] * mb + 1e-30).all(), t
        worst = max(worst, rel_l2(m[t], mo))
    log(f"  worst frame rel L2 {worst:.2e}")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("H,W,n", [(192, 134, 12), (96, 260, 17)])
def test_m2n_runs_match_oracle(H, W, n, prec):
    em = _em()
    p = synth.make_problem("c4", H=H, W=W, n=n, seed=5500 + n)
    x0 = synth.positive_start(p.latent_shape, max(oracle.flat_x0(p.y, p.v, 2), 0.25), seed=5501)
    xg, trg = gpu_run(p.y, p.v, p.psf, 2, 10, x0=x0, precision=getattr(em, prec))
    xo, tro, _ = oracle.run(p.y, p.v, p.psf, x0, 10, 2, trace=True)
    err = rel_l2(xg, xo)
    llerr = float(np.abs(trg - tro).max() / np.abs(tro).max())
    log(f"m2n run {prec} latent {H}x{W} n={n}: rel L2(x) {err:.3e}, loglik rel err {llerr:.3e}")
    assert err <= X_TOL and llerr <= X_TOL and (xg >= 0).all()


@pytest.mark.parametrize("prec", PRECS)
def test_m2n_variants_bitwise_and_autotune(prec):
    import torch
    em = _em()
    p = synth.make_problem("c4", H=160, W=200, n=12, seed=5600)
    x0 = synth.positive_start(p.latent_shape, 2.0, seed=5601)
    prob = em.Problem.make(12, 80, 100, 43, sr=2, precision=getattr(em, prec))
    outs = []
    for fv in range(em._lib.em_variant_count()):
        x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
        ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
        ctx.set_variants(fv, 0)
        ctx.iterate(3)
        ctx.sync()
        outs.append(x.cpu().numpy())
        ctx.close()
        log(f"m2n {prec} variant {fv}: done")
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    xo = oracle.run(p.y, p.v, p.psf, x0, 3, sr=2)
    assert rel_l2(outs[0], xo) <= X_TOL
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
    before = x.clone()
    fv, av, ms = ctx.autotune(1)
    torch.cuda.synchronize()
    assert torch.equal(before, x) and (ms > 0).all()
    ctx.set_variants(fv, 0)
    ctx.iterate(3)
    ctx.sync()
    assert np.array_equal(x.cpu().numpy(), outs[0])
    ctx.close()


@pytest.mark.parametrize("prec", PRECS)
def test_m2n_traced_and_untraced_agree_bitwise(prec):
    """With a log-likelihood trace the forward also forms the FP64 partials; the
    iterates must not change."""
    import torch
    em = _em()
    p = synth.make_problem("c4", H=128, W=132, n=9, seed=5700)
    x0 = synth.positive_start(p.latent_shape, 2.0, seed=5701)
    prob = em.Problem.make(9, 64, 66, 43, sr=2, precision=getattr(em, prec))
    out = []
    for trace in (True, False):
        x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
        ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
        tr = ctx.iterate(4, trace=trace)
        ctx.sync()
        out.append(x.cpu().numpy().copy())
        if trace:
            _, tro, _ = oracle.run(p.y, p.v, p.psf, x0, 4, 2, trace=True)
            assert float(np.abs(tr - tro).max() / np.abs(tro).max()) <= X_TOL
        ctx.close()
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("prec", PRECS)
def test_m2n_student_t_matches_oracle(prec):
    em = _em()
    p = synth.make_problem("c4", H=96, W=112, n=10, seed=5800)
    y, _ = synth.add_trails(p.y, p.v, 5801)
    x0 = synth.positive_start(p.latent_shape, max(oracle.flat_x0(y, p.v, 2), 0.25), seed=5802)
    import torch
    prob = em.Problem.make(10, 48, 56, 43, sr=2, precision=getattr(em, prec), nu=3.0)
    x = torch.empty(p.latent_shape, dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
    tr = ctx.iterate(8, trace=True)
    ctx.sync()
    xg = x.cpu().numpy().astype(np.float64)
    ctx.close()
    xo, tro, _ = oracle.run_t(y, p.v, p.psf, x0, 8, 3.0, 2, trace=True)
    err = rel_l2(xg, xo)
    llerr = float(np.abs(tr - tro).max() / np.abs(tro).max())
    log(f"m2n Student-t {prec}: rel L2(x) {err:.2e}, loglik rel err {llerr:.2e}")
    assert err <= X_TOL and llerr <= X_TOL
