"""Pins of the oracle's design-update steps (filter, OC) against closed forms
and invariants."""
import numpy as np
import pytest

from oracle import topopt


def test_hat_offsets_radius_1_5():
    offs = topopt._offsets(1.5)
    assert len(offs) == 19  # centre, 6 faces, 12 edges (sqrt 2 < 1.5 < sqrt 3)
    W = sum(w for *_, w in offs)
    assert abs(W - (1.5 + 6 * 0.5 + 12 * (1.5 - np.sqrt(2.0)))) < 1e-14


def test_filter_keeps_constants_and_interior_linears():
    n = (7, 6, 5)
    x = np.full(7 * 6 * 5, 0.37)
    assert np.allclose(topopt.density_filter(x, n, 1.5), 0.37, rtol=0, atol=1e-15)
    k, j, i = np.meshgrid(np.arange(5), np.arange(6), np.arange(7), indexing="ij")
    lin = (0.3 * i - 0.2 * j + 0.1 * k + 1.0).ravel()
    out = topopt.density_filter(lin, n, 1.5).reshape(5, 6, 7)
    # symmetric weights reproduce a linear field away from the boundary
    assert np.allclose(out[1:-1, 1:-1, 1:-1], lin.reshape(5, 6, 7)[1:-1, 1:-1, 1:-1], atol=1e-13)


def test_filter_brute_force_tiny():
    n = (3, 2, 2)
    rng = np.random.default_rng(0)
    x = rng.random(12)
    r = 1.5
    cent = [(i, j, k) for k in range(2) for j in range(2) for i in range(3)]
    H = np.zeros((12, 12))
    for e, ce in enumerate(cent):
        for f, cf in enumerate(cent):
            H[e, f] = max(0.0, r - np.linalg.norm(np.subtract(ce, cf)))
    W = H.sum(axis=1)
    assert np.allclose(topopt.density_filter(x, n, r), H @ x / W, atol=1e-15)
    assert np.allclose(topopt.density_filter(x, n, r, transpose=True), H.T @ (x / W), atol=1e-15)


@pytest.mark.parametrize("r", [1.5, 2.0, 2.6])
def test_filter_transpose_is_adjoint(r):
    n = (6, 5, 4)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(120), rng.standard_normal(120)
    lhs = topopt.density_filter(x, n, r) @ y
    rhs = x @ topopt.density_filter(y, n, r, transpose=True)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_oc_volume_and_limits():
    rng = np.random.default_rng(2)
    x = rng.uniform(0.2, 0.5, 500)
    dc = -rng.uniform(0.1, 5.0, 500)
    dv = rng.uniform(0.5, 1.5, 500)
    xn, lam = topopt.oc_update(x, dc, dv, 0.3, move=0.2, eta=0.5, x_min=1e-3)
    assert abs(xn.sum() - 150.0) < 1e-9
    assert np.all(xn >= np.maximum(1e-3, x - 0.2) - 1e-15) and np.all(xn <= np.minimum(1.0, x + 0.2) + 1e-15)
    # inside the limits the OC fixed-point form holds with the returned multiplier
    free = (xn > np.maximum(1e-3, x - 0.2) + 1e-12) & (xn < np.minimum(1.0, x + 0.2) - 1e-12)
    assert free.any()
    assert np.allclose(xn[free], x[free] * np.sqrt(-dc[free] / (lam * dv[free])), rtol=1e-12)


def test_oc_uniform_sensitivity_gives_uniform_design():
    x = np.full(64, 0.3)
    xn, _ = topopt.oc_update(x, -np.ones(64), np.ones(64), 0.3)
    assert np.allclose(xn, 0.3, atol=1e-12)
