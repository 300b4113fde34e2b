"""Serving loop (em_submit / em_poll / em_wait): continuous batching of jobs of
uneven size, frame count and super-resolution factor.

* Each job's result is bitwise the same alone and in a mix (the launch plan of
  a served job depends on its own shape; no reduction crosses jobs).
* Served results match the FP64 oracle within the bar of their precision
  (Gaussian and Student-t jobs).
* Admission respects the HBM budget and the slot count; errors, cancellation.
"""
import numpy as np
import pytest

import oracle
from paper_2302_05804_amd import synth
from tests.gpu_common import log, rel_l2

pytestmark = pytest.mark.gpu


def _em():
    from paper_2302_05804_amd import em
    return em


def _jobs():
    em = _em()
    specs = [  # (recipe, latent H, W, n, sr, precision, iterations, Student-t nu or 0)
        ("c2", 96, 96, 3, 1, em.BF16_SPLIT, 7, 0.0),
        ("c3", 160, 128, 5, 1, em.FP32, 5, 0.0),
        ("c4", 128, 96, 2, 2, em.BF16_SPLIT, 6, 0.0),
        ("c2", 200, 136, 2, 1, em.BF16_SPLIT, 9, 0.0),
        ("c1", 64, 64, 4, 1, em.FP32, 12, 0.0),
        ("c4", 64, 192, 3, 2, em.FP32, 4, 0.0),
        ("c3", 128, 160, 3, 1, em.FP16_SPLIT, 6, 0.0),
        ("c4", 96, 128, 2, 2, em.FP16_SPLIT, 5, 0.0),
        ("c2", 112, 96, 3, 1, em.FP16_SPLIT, 6, 4.0),     # Student-t jobs, with trails
        ("c4", 96, 112, 2, 2, em.FP32, 5, 3.0),
        ("c3", 96, 80, 2, 1, em.BF16_SPLIT, 4, 2.5),
        ("c4", 96, 144, 12, 2, em.FP16_SPLIT, 5, 0.0),    # sr = 2, frames in N
        ("c4", 64, 96, 9, 2, em.FP16_SPLIT, 4, 3.0),
        ("c4", 80, 112, 10, 2, em.BF16_SPLIT, 5, 0.0),    # BF16 split, frames in N
    ]
    out = []
    for k, (rec, H, W, n, sr, prec, it, nu) in enumerate(specs):
        p = synth.make_problem(rec, H=H, W=W, n=n, seed=700 + k)
        if nu:
            p.y, _ = synth.add_trails(p.y, p.v, seed=800 + k)
        prob = em.Problem.make(n, H // sr, W // sr, p.K, sr=sr, precision=prec, nu=nu)
        out.append((p, prob, it))
    return out


def _serve(jobs, budget, slots):
    em = _em()
    srv = em.Server(budget, max_slots=slots)
    ids = [srv.submit(prob, p.y, p.v, p.psf, it) for p, prob, it in jobs]
    res = [srv.wait(j) for j in ids]
    st = srv.stats()
    times = [srv.times(j) for j in ids]
    srv.close()
    return res, st, times


def test_alone_vs_mix_bitwise():
    em = _em()
    jobs = _jobs()
    need = max(em.job_bytes(prob) for _, prob, _ in jobs)
    alone = []
    for job in jobs:
        (r,), st, _ = _serve([job], need + (1 << 20), 1)
        assert st["done"] == 1
        alone.append(r)
    # a budget for about three jobs at a time, four slots: jobs queue and are
    # admitted as others finish
    budget = int(3.2 * need)
    mix, st, times = _serve(jobs, budget, 4)
    log(f"mix stats: {st}")
    assert st["done"] == len(jobs) and st["failed"] == 0
    for (xa, la), (xm, lm) in zip(alone, mix):
        assert np.array_equal(xa, xm)
        assert la == lm
    # continuous batching: some job was admitted after another finished
    admits = sorted(t[1] for t in times)
    dones = sorted(t[2] for t in times)
    assert admits[-1] >= dones[0]


def test_served_results_match_oracle():
    em = _em()
    jobs = _jobs()
    res, st, _ = _serve(jobs, 512 << 20, 8)
    for (p, prob, it), (x, ll) in zip(jobs, res):
        x0 = np.full(p.latent_shape, oracle.flat_x0(p.y, p.v, p.sr), np.float32)
        if prob.nu:
            xo = oracle.run_t(p.y, p.v, p.psf, x0, it, prob.nu, p.sr)
            llo = oracle.loglik_t(p.y, p.v, p.psf, xo, prob.nu, p.sr)
        else:
            xo = oracle.run(p.y, p.v, p.psf, x0, it, p.sr)
            llo = oracle.loglik(p.y, p.v, p.psf, xo, p.sr)
        err = rel_l2(x, xo)
        tol = 1e-5 if prob.precision == em.FP32 else 1e-3
        log(f"job {p.name} {p.latent_shape} sr={p.sr} prec={prob.precision} nu={prob.nu:g}: rel L2 {err:.2e}, "
            f"loglik rel err {abs(ll - llo) / abs(llo):.2e}")
        assert err <= tol
        assert abs(ll - llo) <= 1e-5 * abs(llo)


def test_budget_errors_cancel_and_release():
    em = _em()
    p = synth.make_problem("c2", H=96, W=96, n=2, seed=9)
    prob = em.Problem.make(2, 96, 96, 43)
    need = em.job_bytes(prob)
    srv = em.Server(need + (1 << 20), max_slots=1)
    big = em.Problem.make(8, 512, 512, 43)
    yb = np.zeros((8, 512, 512), np.float32)
    with pytest.raises(em.EMError) as ei:
        srv.submit(big, yb, yb + 1, np.ones((8, 43, 43), np.float32), 3)
    assert ei.value.code == em.ENOMEM
    bad_v = p.v.copy()
    bad_v[0, 3, 3] = 0.0
    j_bad = srv.submit(prob, p.y, bad_v, p.psf, 3)
    j1 = srv.submit(prob, p.y, p.v, p.psf, 40)
    j2 = srv.submit(prob, p.y, p.v, p.psf, 5)     # queued behind j1 (one slot)
    srv.cancel(j2)
    with pytest.raises(em.EMError) as ei:
        srv.wait(j_bad)
    assert ei.value.code == em.EINVAL
    x1, ll1 = srv.wait(j1)
    assert np.isfinite(x1).all() and (x1 >= 0).all()
    with pytest.raises(em.EMError) as ei:
        srv.wait(j2)
    assert ei.value.code == em.ECANCELED
    j0 = srv.submit(prob, p.y, p.v, p.psf, 0)      # zero iterations: the flat start
    x0, _ = srv.wait(j0)
    assert np.allclose(x0, oracle.flat_x0(p.y, p.v), rtol=1e-6)
    srv.release(j1)
    with pytest.raises(em.EMError):
        srv.poll(j1)
    st = srv.stats()
    assert st["arena_bytes_in_use"] == 0 and st["active"] == 0
    srv.close()


def test_concurrent_clients_match_one_client_bitwise():
    """Server calls are thread-safe: four client threads submit, poll and wait
    on their own jobs while a fifth reads the statistics; every result is
    bitwise the one a single client gets for the same job."""
    import threading
    import time

    em = _em()
    jobs = _jobs()[:8]
    ref, _, _ = _serve(jobs, 512 << 20, 4)
    srv = em.Server(512 << 20, max_slots=4)
    out = [None] * len(jobs)
    errors = []
    done = threading.Event()

    def client(ks):
        try:
            ids = [(k, srv.submit(jobs[k][1], jobs[k][0].y, jobs[k][0].v, jobs[k][0].psf,
                                  jobs[k][2])) for k in ks]
            for k, j in ids:
                deadline = time.time() + 120
                while srv.poll(j) is None:
                    assert time.time() < deadline, f"job {k} still pending"
                    time.sleep(0.002)
                out[k] = srv.wait(j)
        except Exception as e:   # reported in the main thread
            errors.append(e)

    def watcher():
        try:
            while not done.is_set():
                st = srv.stats()
                assert st["active"] <= 4 and st["failed"] == 0
                time.sleep(0.001)
        except Exception as e:
            errors.append(e)

    threads = [threading.Thread(target=client, args=(list(range(c, len(jobs), 4)),))
               for c in range(4)]
    w = threading.Thread(target=watcher)
    w.start()
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    done.set()
    w.join(timeout=30)
    st = srv.stats()
    srv.close()
    assert not errors, errors
    assert st["done"] == len(jobs) and st["failed"] == 0
    for k, ((xa, la), res) in enumerate(zip(ref, out)):
        assert res is not None, k
        assert np.array_equal(xa, res[0]) and la == res[1], k



def test_pinned_and_pageable_staging_bitwise():
    """A job's inputs go through the server's pinned staging area (a quarter of
    the budget) when it has room, else through pageable memory; the result is
    bitwise the same.  Here job A runs (one slot), job B waits behind it holding
    most of the staging area, so job C is staged in pageable memory; C alone on
    a fresh server is staged in pinned memory."""
    import time
    em = _em()
    al = lambda b: (b + 255) // 256 * 256
    pa = synth.make_problem("c1", H=64, W=64, n=4, seed=7)
    prob_a = em.Problem.make(4, 64, 64, pa.K, precision=em.FP32)
    pb = synth.make_problem("c2", H=256, W=256, n=12, seed=8)
    prob_b = em.Problem.make(12, 256, 256, pb.K, precision=em.FP32)
    for k in (1, 2, 6, 8):            # FP32, BF16 sr = 2, FP16, FP16 Student-t
        pc, prob_c, it = _jobs()[k]
        staged = al(pb.y.nbytes + pb.v.nbytes) + al(pc.y.nbytes + pc.v.nbytes)
        budget = 4 * staged - 1024
        assert max(em.job_bytes(q) for q in (prob_a, prob_b, prob_c)) <= budget
        srv = em.Server(budget, max_slots=1)
        ja = srv.submit(prob_a, pa.y, pa.v, pa.psf, 3000)
        t0 = time.time()
        while srv.stats()["active"] == 0:
            assert time.time() - t0 < 60
            time.sleep(0.001)
        srv.submit(prob_b, pb.y, pb.v, pb.psf, 2)
        jc = srv.submit(prob_c, pc.y, pc.v, pc.psf, it)
        st_mix = srv.staging()
        xc, llc = srv.wait(jc)
        srv.wait(ja)
        srv.close()
        srv = em.Server(512 << 20, max_slots=1)
        xs, lls = srv.wait(srv.submit(prob_c, pc.y, pc.v, pc.psf, it))
        st_alone = srv.staging()
        srv.close()
        log(f"job {pc.name} {pc.latent_shape} sr={pc.sr}: staging in the mix {st_mix}, "
            f"alone {st_alone}")
        assert st_mix["pinned_jobs"] == 2 and st_mix["pageable_jobs"] == 1
        assert st_alone["pinned_jobs"] == 1 and st_alone["pageable_jobs"] == 0
        assert np.array_equal(xc, xs) and llc == lls
