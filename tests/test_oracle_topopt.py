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


# --- MMA (Svanberg) -----------------------------------------------------------

def _mma_case(N=40, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.2, 0.8, N)
    xold1 = np.clip(x + rng.uniform(-0.05, 0.05, N), 1e-3, 1)
    xold2 = np.clip(xold1 + rng.uniform(-0.05, 0.05, N), 1e-3, 1)
    low, upp = x - 0.3, x + 0.3
    df0 = -np.exp(rng.standard_normal(N))
    dv = rng.uniform(0.5, 1.5, N)
    return x, xold1, xold2, low, upp, df0, dv


def test_mma_asymptote_rules():
    x, xold1, xold2, low, upp, _, _ = _mma_case()
    lo, up = topopt.mma_asymptotes(0, x, xold1, xold2, low, upp, 0.0, 1.0)
    assert np.allclose(lo, x - 0.5) and np.allclose(up, x + 0.5)
    lo, up = topopt.mma_asymptotes(5, x, xold1, xold2, low, upp, 0.0, 1.0)
    osc = (x - xold1) * (xold1 - xold2) < 0
    mono = (x - xold1) * (xold1 - xold2) > 0
    want_lo = np.clip(x - np.where(osc, 0.7, np.where(mono, 1.2, 1.0)) * (xold1 - low), x - 10, x - 0.01)
    want_up = np.clip(x + np.where(osc, 0.7, np.where(mono, 1.2, 1.0)) * (upp - xold1), x + 0.01, x + 10)
    assert np.array_equal(lo, want_lo) and np.array_equal(up, want_up)
    assert osc.any() and mono.any()


@pytest.mark.parametrize("seed,shift", [(0, -0.05), (1, -0.02), (2, 5.0), (3, -0.3)])
def test_mma_subproblem_is_solved(seed, shift):
    """The update solves the convex approximate problem (objective + c y +
    y^2 / 2, approximate constraint <= y, move limits): the Karush-Kuhn-Tucker
    conditions hold, which for a convex problem certify the global minimum.
    Volume targets just below the current design (active constraint), far
    above it (the convex approximation of the volume stays below the target
    over the whole move box: inactive, lam = 0) and far below (unreachable:
    y > 0)."""
    x, xold1, xold2, low, upp, df0, dv = _mma_case(seed=seed)
    N, span, c = x.size, 1.0 - 1e-3, topopt.MMA_C
    vf = float(dv @ x) / N + shift
    xn, lo, up, lam = topopt.mma_update(3, x, xold1, xold2, low, upp, df0, dv, vf, move=0.2)
    alpha = np.maximum.reduce([np.full(N, 1e-3), lo + 0.1 * (x - lo), x - 0.2 * span])
    beta = np.minimum.reduce([np.full(N, 1.0), up - 0.1 * (up - x), x + 0.2 * span])
    p0, q0 = topopt.mma_terms(x, lo, up, df0, 1e-3, 1.0)
    p1, q1 = topopt.mma_terms(x, lo, up, dv / N, 1e-3, 1.0)
    y = max(0.0, lam - c)
    _, g = topopt.mma_subproblem_objective(xn, x, lo, up, df0, dv, vf)
    # stationarity in x: zero derivative inside the limits, the right sign at them
    d = (p0 + lam * p1) / (up - xn) ** 2 - (q0 + lam * q1) / (xn - lo) ** 2
    scale = (p0 + lam * p1) / (up - xn) ** 2 + (q0 + lam * q1) / (xn - lo) ** 2
    at_lo, at_hi = xn <= alpha, xn >= beta
    inner = ~(at_lo | at_hi)
    assert np.all(alpha <= xn) and np.all(xn <= beta)
    assert np.all(np.abs(d[inner]) <= 1e-12 * scale[inner])
    assert np.all(d[at_lo] >= -1e-12 * scale[at_lo]) and np.all(d[at_hi] <= 1e-12 * scale[at_hi])
    # stationarity in y, feasibility, complementarity
    assert (y == 0.0 and lam <= c) or abs(c + y - lam) <= 1e-12 * lam
    assert g <= y + 1e-10
    assert lam == 0.0 or abs(g - y) <= 1e-9
    if shift > 0:
        assert lam == 0.0 and g < 0
    elif shift == -0.3:
        assert y > 0.0
    else:
        assert 0.0 < lam < c


def test_mma_converges_to_the_closed_form_optimum():
    """min sum c_e / x_e subject to mean(x) = vf has the optimum
    x_e = vf N sqrt(c_e) / sum sqrt(c) (Lagrange: c_e / x_e^2 constant);
    MMA iterations with the exact gradient reach it."""
    rng = np.random.default_rng(3)
    N, vf = 50, 0.4
    c = rng.uniform(0.5, 2.0, N)
    x_star = vf * N * np.sqrt(c) / np.sqrt(c).sum()
    assert x_star.min() > 1e-3 and x_star.max() < 1.0
    x = np.full(N, vf)
    xold1 = xold2 = x.copy()
    low, upp = x - 0.5, x + 0.5
    dv = np.ones(N)
    for it in range(60):
        xn, low, upp, lam = topopt.mma_update(it, x, xold1, xold2, low, upp, -c / x ** 2, dv, vf)
        xold2, xold1, x = xold1, x, xn
    assert np.abs(x - x_star).max() <= 1e-6
