"""The seeded generators produce the workload shapes and distributions."""
import numpy as np

from paper_2302_05804_amd import synth


def test_c1_shapes_and_determinism():
    a = synth.make_problem("c1")
    b = synth.make_problem("c1")
    assert a.y.shape == (4, 128, 128) and a.psf.shape == (4, 15, 15) and a.sr == 1
    assert np.array_equal(a.y, b.y) and np.array_equal(a.psf, b.psf)
    assert a.y.dtype == np.float32 and a.v.dtype == np.float32
    np.testing.assert_allclose(a.psf.sum(axis=(1, 2)), 1.0, rtol=1e-5)
    assert (a.v >= 10.0).all() and (a.x_true >= 0).all()
    assert a.n_iter == 30


def test_c2_scaled_masks_and_psf():
    p = synth.make_problem("c2", H=256, W=192, n=3)
    assert p.y.shape == (3, 256, 192) and p.K == 43
    masked = ~np.isfinite(p.v)
    assert np.isnan(p.y[masked]).all() and np.isfinite(p.y[~masked]).all()
    frac = masked.mean()
    assert 0.01 < frac < 0.03
    # PSF peak at the centre
    for t in range(3):
        iy, ix = np.unravel_index(np.argmax(p.psf[t]), p.psf[t].shape)
        assert abs(iy - 21) <= 1 and abs(ix - 21) <= 1


def test_c3_streak_masks_scaled():
    p = synth.make_problem("c3", H=512, W=512, n=2)
    frac = (~np.isfinite(p.v)).mean()
    assert 0.004 < frac < 0.02


def test_c4_super_resolution_shapes():
    p = synth.make_problem("c4", H=256, W=128, n=2)
    assert p.sr == 2 and p.y.shape == (2, 128, 64) and p.latent_shape == (256, 128)


def test_serving_stream():
    jobs = synth.serving_stream(50, rate=2.0)
    assert all(64 <= j.frame_side <= 2048 and j.frame_side % 64 == 0 for j in jobs)
    assert all(4 <= j.n <= 33 and j.sr in (1, 2) and 50 <= j.n_iter <= 200 for j in jobs)
    arr = [j.arrival for j in jobs]
    assert arr == sorted(arr)
