"""Parity of the BF16 matrix-core path (hi+lo split operands) with the FP64 oracle.

Error model of one correlation output o = sum_k g_k in_k computed with split
operands v = hi + lo (+ delta): each product loses the lo.lo term and the
representation remainders, at most 3 * 2^-16 |g_k in_k|; FP32 accumulation adds
at most ~(#terms) 2^-24 sum |g_k in_k| in the worst case.  The operator tests
bound |o_gpu - o| <= 1e-4 * sum_k |g_k||in_k| element by element (computed by
the oracle on absolute values).  Whole EM runs must stay within rel L2 1e-3 of
the oracle's iterate (the accuracy bar of the mixed-precision form).
"""
import numpy as np
import pytest

import oracle
from paper_2302_05804_amd import synth
from tests.gpu_common import gpu_run, log, rel_l2, to_dev

pytestmark = pytest.mark.gpu

OP_EPS = 1e-4
SPLIT_X_TOL = 1e-3


def _em():
    from paper_2302_05804_amd import em
    return em


@pytest.mark.parametrize("K,h,w,n", [(43, 150, 131, 2), (15, 70, 260, 3), (43, 256, 128, 1),
                                     (7, 33, 40, 2), (43, 5, 3, 1), (43, 129, 257, 1)])
def test_split_operators_elementwise_bound(K, h, w, n):
    em = _em()
    log(f"mfma operators K={K} {h}x{w} n={n}")
    rng = np.random.default_rng(K * 7 + h)
    psf = rng.uniform(0, 1, (n, K, K)).astype(np.float32)
    psf /= psf.sum(axis=(1, 2), keepdims=True)
    x = rng.gamma(0.5, 200.0, (h, w)).astype(np.float32)
    r = rng.normal(0, 1, (n, h, w)).astype(np.float32)
    p = em.Problem.make(n, h, w, K, precision=em.BF16_SPLIT)
    m = em.forward_op(p, to_dev(psf), to_dev(x)).cpu().numpy()
    s = em.adjoint_op(p, to_dev(psf), to_dev(r)).cpu().numpy()
    for t in range(n):
        mo = oracle.forward(psf[t], x)
        so = oracle.adjoint(psf[t], r[t])
        mb = oracle.forward(np.abs(psf[t]), np.abs(x))
        sb = oracle.adjoint(np.abs(psf[t]), np.abs(r[t]))
        assert (np.abs(m[t] - mo) <= OP_EPS * mb + 1e-30).all()
        assert (np.abs(s[t] - so) <= OP_EPS * sb + 1e-30).all()
        log(f"  t={t}: rel L2 fwd {rel_l2(m[t], mo):.2e} adj {rel_l2(s[t], so):.2e}")


def test_plain_bf16_operator_is_coarser():
    em = _em()
    rng = np.random.default_rng(5)
    psf = rng.uniform(0, 1, (1, 43, 43)).astype(np.float32)
    psf /= psf.sum()
    x = rng.uniform(0, 100, (96, 96)).astype(np.float32)
    ps = em.Problem.make(1, 96, 96, 43, precision=em.BF16_SPLIT)
    pb = em.Problem.make(1, 96, 96, 43, precision=em.BF16)
    mo = oracle.forward(psf[0], x)
    es = rel_l2(em.forward_op(ps, to_dev(psf), to_dev(x)).cpu().numpy()[0], mo)
    eb = rel_l2(em.forward_op(pb, to_dev(psf), to_dev(x)).cpu().numpy()[0], mo)
    log(f"forward rel L2: split {es:.2e}, plain bf16 {eb:.2e}")
    assert es < 1e-5 and eb > 10 * es


def _run_both(prob, n_iter, x0, precision):
    em = _em()
    xg, trg = gpu_run(prob.y, prob.v, prob.psf, prob.sr, n_iter, x0=x0, precision=precision)
    xo, tro, _ = oracle.run(prob.y, prob.v, prob.psf, x0, n_iter, prob.sr, trace=True)
    err = rel_l2(xg, xo)
    llerr = float(np.abs(trg - tro).max() / np.abs(tro).max())
    return err, llerr, xg, trg


def test_c1_split_full_run():
    em = _em()
    p = synth.make_problem("c1")
    x0 = np.full(p.latent_shape, oracle.flat_x0(p.y, p.v), np.float32)
    err, llerr, xg, trg = _run_both(p, p.n_iter, x0, em.BF16_SPLIT)
    log(f"c1 bf16-split: rel L2(x) {err:.3e}, loglik rel err {llerr:.3e}")
    assert err <= SPLIT_X_TOL
    assert (xg >= 0).all()
    assert (np.diff(trg) >= -1e-7 * np.abs(trg[1:])).all()


def test_c2_recipe_split_ragged():
    em = _em()
    p = synth.make_problem("c2", H=200, W=173, n=3)
    x0 = synth.positive_start(p.latent_shape, max(oracle.flat_x0(p.y, p.v), 1.0), seed=7)
    err, llerr, xg, _ = _run_both(p, 10, x0, em.BF16_SPLIT)
    log(f"c2-ragged bf16-split: rel L2(x) {err:.3e}, loglik rel err {llerr:.3e}")
    assert err <= SPLIT_X_TOL and (xg >= 0).all()


def test_c3_recipe_split_multi_tile():
    em = _em()
    p = synth.make_problem("c3", H=300, W=260, n=4)
    x0 = synth.positive_start(p.latent_shape, max(oracle.flat_x0(p.y, p.v), 1.0), seed=8)
    err, llerr, xg, _ = _run_both(p, 6, x0, em.BF16_SPLIT)
    log(f"c3-tiles bf16-split: rel L2(x) {err:.3e}, loglik rel err {llerr:.3e}")
    assert err <= SPLIT_X_TOL and (xg >= 0).all()


def test_split_deterministic():
    em = _em()
    p = synth.make_problem("c2", H=140, W=150, n=3)
    x0 = synth.positive_start(p.latent_shape, 20.0, seed=6)
    a, ta = gpu_run(p.y, p.v, p.psf, 1, 4, x0=x0, precision=em.BF16_SPLIT)
    b, tb = gpu_run(p.y, p.v, p.psf, 1, 4, x0=x0, precision=em.BF16_SPLIT)
    assert np.array_equal(a, b) and np.array_equal(ta, tb)


# ---------------------------------------------------------------------------
# super-resolution (sr = 2, Eq. (3)) on the matrix cores
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K,hf,wf,n", [(43, 75, 66, 2), (43, 64, 64, 1), (15, 40, 70, 3),
                                       (43, 17, 130, 1), (43, 3, 2, 1), (43, 130, 97, 2)])
def test_split_sr2_operators_elementwise_bound(K, hf, wf, n):
    em = _em()
    log(f"mfma sr=2 operators K={K} frame {hf}x{wf} n={n}")
    rng = np.random.default_rng(K * 11 + hf)
    psf = rng.uniform(0, 1, (n, K, K)).astype(np.float32)
    psf /= psf.sum(axis=(1, 2), keepdims=True)
    x = rng.gamma(0.5, 200.0, (2 * hf, 2 * wf)).astype(np.float32)
    r = rng.normal(0, 1, (n, hf, wf)).astype(np.float32)
    p = em.Problem.make(n, hf, wf, K, sr=2, precision=em.BF16_SPLIT)
    m = em.forward_op(p, to_dev(psf), to_dev(x)).cpu().numpy()
    s = em.adjoint_op(p, to_dev(psf), to_dev(r)).cpu().numpy()
    for t in range(n):
        mo = oracle.forward(psf[t], x, 2)
        so = oracle.adjoint(psf[t], r[t], 2)
        mb = oracle.forward(np.abs(psf[t]), np.abs(x), 2)
        sb = oracle.adjoint(np.abs(psf[t]), np.abs(r[t]), 2)
        assert (np.abs(m[t] - mo) <= OP_EPS * mb + 1e-30).all()
        assert (np.abs(s[t] - so) <= OP_EPS * sb + 1e-30).all()
        log(f"  t={t}: rel L2 fwd {rel_l2(m[t], mo):.2e} adj {rel_l2(s[t], so):.2e}")


def test_c4_recipe_split_sr2_runs():
    em = _em()
    p = synth.make_problem("c4", H=192, W=134, n=3)
    x0 = synth.positive_start(p.latent_shape, max(oracle.flat_x0(p.y, p.v, 2), 0.25), seed=9)
    err, llerr, xg, trg = _run_both(p, 10, x0, em.BF16_SPLIT)
    log(f"c4-sr2 bf16-split: rel L2(x) {err:.3e}, loglik rel err {llerr:.3e}")
    assert err <= SPLIT_X_TOL and (xg >= 0).all()
    assert (np.diff(trg) >= -1e-7 * np.abs(trg[1:])).all()
    p2 = synth.make_problem("c4", H=300, W=260, n=2, seed=4401)
    x02 = synth.positive_start(p2.latent_shape, max(oracle.flat_x0(p2.y, p2.v, 2), 0.25), seed=10)
    err2, _, xg2, _ = _run_both(p2, 5, x02, em.BF16_SPLIT)
    log(f"c4-sr2 multi-tile bf16-split: rel L2(x) {err2:.3e}")
    assert err2 <= SPLIT_X_TOL


def test_sr2_every_variant_matches_oracle():
    import torch
    em = _em()
    p = synth.make_problem("c4", H=260, W=200, n=2, seed=4402)
    x0 = synth.positive_start(p.latent_shape, 2.0, seed=13)
    xo = oracle.run(p.y, p.v, p.psf, x0, 3, sr=2)
    prob = em.Problem.make(2, 130, 100, 43, sr=2, precision=em.BF16_SPLIT)
    nv = em._lib.em_variant_count()
    for fv in range(nv):
        for av in range(nv):
            x = torch.empty((260, 200), dtype=torch.float32, device="cuda")
            ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
            ctx.set_variants(fv, av)
            ctx.iterate(3)
            ctx.sync()
            err = rel_l2(x.cpu().numpy(), xo)
            ctx.close()
            log(f"sr2 variant fwd={fv} adj={av}: rel L2 {err:.2e}")
            assert err <= SPLIT_X_TOL


def test_every_variant_and_autotune_match_oracle():
    import torch
    em = _em()
    p = synth.make_problem("c3", H=260, W=300, n=3)
    x0 = synth.positive_start(p.latent_shape, max(oracle.flat_x0(p.y, p.v), 1.0), seed=12)
    xo = oracle.run(p.y, p.v, p.psf, x0, 4)
    prob = em.Problem.make(3, 260, 300, 43, precision=em.BF16_SPLIT)
    nv = em._lib.em_variant_count()
    assert nv >= 2
    outs = []
    for fv in range(nv):
        for av in range(nv):
            x = torch.empty((260, 300), dtype=torch.float32, device="cuda")
            ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
            ctx.set_variants(fv, av)
            ctx.iterate(4)
            ctx.sync()
            xg = x.cpu().numpy()
            ctx.close()
            err = rel_l2(xg, xo)
            log(f"variant fwd={fv} adj={av}: rel L2 {err:.2e}")
            assert err <= SPLIT_X_TOL
            outs.append(xg)
    # autotune leaves the iterate alone and picks valid variants
    x = torch.empty((260, 300), dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
    before = x.clone()
    f, a, ms = ctx.autotune(2)
    assert torch.equal(before, x)
    assert 0 <= f < nv and 0 <= a < nv and (ms > 0).all()
    ctx.iterate(4)
    ctx.sync()
    assert rel_l2(x.cpu().numpy(), xo) <= SPLIT_X_TOL
    ctx.close()


def test_sr2_autotune_then_iterate_matches_oracle():
    """Autotuning an sr = 2 job times its forward kernel on the frame grid and
    its adjoint on the latent grid; the iterate is untouched and the tuned
    iteration still matches the oracle."""
    import torch
    em = _em()
    p = synth.make_problem("c4", H=256, W=192, n=3, seed=4403)
    x0 = synth.positive_start(p.latent_shape, 2.0, seed=14)
    xo = oracle.run(p.y, p.v, p.psf, x0, 3, sr=2)
    prob = em.Problem.make(3, 128, 96, 43, sr=2, precision=em.BF16_SPLIT)
    x = torch.empty((256, 192), dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(p.y), to_dev(p.v), to_dev(p.psf), x, x0=to_dev(x0))
    before = x.clone()
    f, a, ms = ctx.autotune(2)
    torch.cuda.synchronize()
    assert torch.equal(before, x) and (ms > 0).all()
    ctx.iterate(3)
    ctx.sync()
    err = rel_l2(x.cpu().numpy(), xo)
    log(f"sr2 autotuned (fwd {f}, adj {a}): rel L2 {err:.2e}")
    assert err <= SPLIT_X_TOL
    ctx.close()


def test_split_iteration_keeps_full_lo_for_broad_psf():
    """The BF16 split iteration keeps only the hi x hi product outside the 21
    central kernel rows, and only for jobs whose every PSF keeps at most 1/16 of
    its mass outside them.  Here frame 2 is flat over the 43 x 43 stamp (51% of its mass
    outside) and every tap's lo part is 0.99 * 2^-8 of its hi part, so dropping
    it would move B by 6e-4 to 8e-4 relative (frame 2 carries a third of B);
    with the full lo part (and all operands positive) each element of B stays
    within 1e-4 of the oracle's and each of Dn within 2e-4 (two operator
    passes)."""
    import torch
    em = _em()
    n, h, w, K = 3, 150, 141, 43
    rng = np.random.default_rng(44)
    a = np.arange(K) - K // 2
    g = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / 8.0)
    psf = np.empty((n, K, K), np.float32)
    psf[0] = g / g.sum()
    psf[1] = np.roll(g, (1, -2), (0, 1)) / g.sum()
    psf[2] = np.float32(2.0 ** -11 * (1.0 + 0.99 * 2.0 ** -8))
    y = rng.uniform(10.0, 100.0, (n, h, w)).astype(np.float32)
    v = rng.uniform(1.0, 2.0, (n, h, w)).astype(np.float32)
    x0 = rng.uniform(5.0, 50.0, (h, w)).astype(np.float32)
    prob = em.Problem.make(n, h, w, K, precision=em.BF16_SPLIT)
    x = torch.empty((h, w), dtype=torch.float32, device="cuda")
    ctx = em.Context(prob, to_dev(y), to_dev(v), to_dev(psf), x, x0=to_dev(x0))
    B, Dn = ctx.terms()
    ctx.sync()
    B, Dn = B.cpu().numpy(), Dn.cpu().numpy()
    ctx.close()
    Bo = oracle.numerator(y, v, psf)
    Dno = oracle.denominator(y, v, psf, x0)
    eb = float(np.max(np.abs(B - Bo) / Bo))
    ed = float(np.max(np.abs(Dn - Dno) / Dno))
    log(f"broad PSF bf16-split terms: max rel err B {eb:.2e}, Dn {ed:.2e}")
    assert eb <= 1e-4 and ed <= 2e-4
