"""Pins of the oracle's grid transfer (CPU only)."""
import numpy as np

from oracle import interp


def _q1_value(t, nc, pt):
    """Value of the Q1 function with nodal values t (on an nc mesh of the unit box) at pt."""
    ncx, ncy, ncz = nc
    t = t.reshape(ncz + 1, ncy + 1, ncx + 1)
    out = 0.0
    idx, w = [], []
    for c, n in zip(pt, (ncx, ncy, ncz)):
        s = c * n
        i = min(int(np.floor(s)), n - 1)
        idx.append(i)
        w.append(s - i)
    for az in (0, 1):
        for ay in (0, 1):
            for ax in (0, 1):
                f = (w[0] if ax else 1 - w[0]) * (w[1] if ay else 1 - w[1]) * (w[2] if az else 1 - w[2])
                out += f * t[idx[2] + az, idx[1] + ay, idx[0] + ax]
    return out


def test_prolongation_is_the_q1_embedding():
    nc = (3, 4, 5)
    rng = np.random.default_rng(0)
    tc = rng.standard_normal((nc[2] + 1, nc[1] + 1, nc[0] + 1))
    tf = interp.prolong_nodal(tc, nc)
    # coarse nodes keep their values
    assert np.array_equal(tf[::2, ::2, ::2], tc)
    nf = tuple(2 * n for n in nc)
    for pt in rng.uniform(size=(50, 3)):
        assert abs(_q1_value(tf, nf, pt) - _q1_value(tc, nc, pt)) <= 1e-13


def test_prolongation_exact_on_trilinear_polynomials():
    nc = (4, 4, 4)
    z, y, x = np.meshgrid(*(np.arange(n + 1) / n for n in nc[::-1]), indexing="ij")
    zf, yf, xf = np.meshgrid(*(np.arange(2 * n + 1) / (2 * n) for n in nc[::-1]), indexing="ij")
    for fn in (lambda x, y, z: 1 + 0 * x, lambda x, y, z: x + 2 * y - z, lambda x, y, z: x * y * z + y * z):
        tf = interp.prolong_nodal(fn(x, y, z), nc)
        assert np.abs(tf - fn(xf, yf, zf)).max() <= 1e-14


def test_injection_preserves_values_and_mass():
    nc = (3, 2, 4)
    rc = np.random.default_rng(1).uniform(size=(4, 2, 3))
    rf = interp.inject_element(rc, nc)
    assert rf.shape == (8, 4, 6)
    assert np.array_equal(rf[1::2, 0::2, 1::2], rc)
    assert abs(rf.sum() / 8 - rc.sum()) <= 1e-14 * rc.sum()
