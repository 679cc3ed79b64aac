"""Seeded input generators: determinism, shapes and the stated statistics."""
import numpy as np

import synth


def test_uniform_noise_field():
    r = synth.uniform_noise_rho(16, 0)
    assert r.shape == (16, 16, 16)
    assert r.min() >= 0.25 and r.max() <= 0.35
    assert np.array_equal(r, synth.uniform_noise_rho(16, 0))
    assert not np.array_equal(r, synth.uniform_noise_rho(16, 1))


def test_grf_threshold_volume_fraction_and_values():
    r = synth.grf_rho(32, 8, seed=0)
    assert set(np.unique(r)) == {1e-3, 1.0}
    vf = (r == 1.0).mean()
    assert abs(vf - 0.4) <= 1.0 / r.size + 1e-12
    assert np.array_equal(r, synth.grf_rho(32, 8, seed=0))


def test_grf_correlation_length():
    """Sample covariance at lag ell/2 and ell follows exp(-r^2 / (2 ell^2))."""
    ell = 6
    w = synth.grf_raw(96, ell, seed=3)
    w = (w - w.mean()) / w.std()
    for lag in (ell // 2, ell):
        c = np.mean(w * np.roll(w, lag, axis=2))
        assert abs(c - np.exp(-lag ** 2 / (2 * ell ** 2))) < 0.08


def test_dirichlet_patch():
    m = synth.dirichlet_patch_mask(16, 16, 16)
    assert m.shape == (17, 17, 17)
    assert m.sum() == 9 and m[0].sum() == 9 and m[1:].sum() == 0
    assert synth.dirichlet_patch_mask(128, 128, 128).sum() == 625
    assert synth.dirichlet_patch_mask(256, 256, 256).sum() == 2601
    assert synth.dirichlet_patch_mask(8, 8, 8).sum() == 1
