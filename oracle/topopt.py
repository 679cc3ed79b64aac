"""TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): plain NumPy versions of
the design-update steps around the solve, for parity tests of the HIP kernels.

* density filter with linear hat weights w(e,f) = max(0, r - |c_e - c_f|)
  (element centres, element units), normalised by W_e = sum_f w(e,f) over the
  elements inside the mesh, and its adjoint;
* optimality-criteria update x_new = clamp(x (-dc/(lambda dv))^eta, ...) with the
  volume multiplier found by bisection (the textbook OC scheme; the paper's
  optimiser of section 2.3 is MMA, replaced here by OC).
"""
from __future__ import annotations

import itertools

import numpy as np


def _offsets(r):
    R = int(np.floor(r))
    if R >= r:
        R -= 1
    out = []
    for dz, dy, dx in itertools.product(range(-R, R + 1), repeat=3):
        w = r - np.sqrt(dx * dx + dy * dy + dz * dz)
        if w > 0:
            out.append((dx, dy, dz, w))
    return out


def _shifted(a, dx, dy, dz):
    """b[k,j,i] = a[k+dz, j+dy, i+dx] where inside, else 0; and the inside mask."""
    nz, ny, nx = a.shape
    b = np.zeros_like(a)
    m = np.zeros(a.shape, dtype=bool)
    zs, ys, xs = slice(max(0, -dz), min(nz, nz - dz)), slice(max(0, -dy), min(ny, ny - dy)), slice(max(0, -dx), min(nx, nx - dx))
    zt, yt, xt = slice(max(0, dz), min(nz, nz + dz)), slice(max(0, dy), min(ny, ny + dy)), slice(max(0, dx), min(nx, nx + dx))
    b[zs, ys, xs] = a[zt, yt, xt]
    m[zs, ys, xs] = True
    return b, m


def filter_weight_sums(n, r):
    nx, ny, nz = n
    W = np.zeros((nz, ny, nx))
    ones = np.ones((nz, ny, nx))
    for dx, dy, dz, w in _offsets(r):
        _, m = _shifted(ones, dx, dy, dz)
        W += w * m
    return W


def density_filter(x, n, r, transpose=False):
    nx, ny, nz = n
    a = np.asarray(x, dtype=np.float64).reshape(nz, ny, nx)
    W = filter_weight_sums(n, r)
    src = a / W if transpose else a
    out = np.zeros_like(a)
    for dx, dy, dz, w in _offsets(r):
        b, _ = _shifted(src, dx, dy, dz)
        out += w * b
    return (out if transpose else out / W).ravel()


def oc_update(x, dc, dv, volume_fraction, move=0.2, eta=0.5, x_min=1e-3, tol=1e-13):
    """Returns (x_new, lambda) with sum x_new = volume_fraction * len(x)."""
    x = np.asarray(x, dtype=np.float64)
    B0 = np.maximum(0.0, -np.asarray(dc, dtype=np.float64)) / np.asarray(dv, dtype=np.float64)
    lo_b, hi_b = np.maximum(x_min, x - move), np.minimum(1.0, x + move)
    target = volume_fraction * len(x)

    def new(lam):
        return np.clip(x * (B0 / lam) ** eta, lo_b, hi_b)

    # bisection on log(lambda): the volume is non-increasing in lambda
    a, b = np.log(1e-40), np.log(1e40)
    while b - a > tol:
        m = 0.5 * (a + b)
        if new(np.exp(m)).sum() > target:
            a = m
        else:
            b = m
    lam = np.exp(0.5 * (a + b))
    return new(lam), lam


# ---------------------------------------------------------------------------
# Method of moving asymptotes (Svanberg 1987, "The method of moving asymptotes
# - a new method for structural optimization"; the conventions of his 2007 note
# "MMA and GCMMA - two methods for nonlinear optimization"), the optimiser the
# paper's section 2.3 uses, for one linear volume constraint
#     f1(x) = dv . x / N - vf <= 0,   x_min <= x <= x_max.
# Each update builds the separable convex approximation at x (asymptotes L, U
# moved by the sign pattern of the last two steps), bounds the step by
# alpha, beta, and solves the approximate problem through its dual: for a
# multiplier lam >= 0 every x_e minimises its own convex term in closed form,
# and the dual derivative (the constraint value of that x minus the elastic
# variable y = max(0, lam - c)) is non-increasing in lam, so lam follows by
# bisection.

MMA_ASYINIT, MMA_ASYINCR, MMA_ASYDECR, MMA_ALBEFA, MMA_RAA0, MMA_C = 0.5, 1.2, 0.7, 0.1, 1e-5, 1000.0


def mma_asymptotes(it, x, xold1, xold2, low, upp, x_min=0.0, x_max=1.0):
    """Lower and upper asymptotes of update number `it` (0-based)."""
    span = x_max - x_min
    if it < 2:
        return x - MMA_ASYINIT * span, x + MMA_ASYINIT * span
    sgn = (x - xold1) * (xold1 - xold2)
    gam = np.where(sgn < 0, MMA_ASYDECR, np.where(sgn > 0, MMA_ASYINCR, 1.0))
    lo = x - gam * (xold1 - low)
    up = x + gam * (upp - xold1)
    lo = np.clip(lo, x - 10.0 * span, x - 0.01 * span)
    up = np.clip(up, x + 0.01 * span, x + 10.0 * span)
    return lo, up


def mma_terms(x, lo, up, grad, x_min=0.0, x_max=1.0):
    """p, q of one function's approximation sum_e p_e/(U_e - x_e) + q_e/(x_e - L_e) + r."""
    reg = MMA_RAA0 / (x_max - x_min)
    gp, gm = np.maximum(grad, 0.0), np.maximum(-grad, 0.0)
    p = (up - x) ** 2 * (1.001 * gp + 0.001 * gm + reg)
    q = (x - lo) ** 2 * (0.001 * gp + 1.001 * gm + reg)
    return p, q


def mma_update(it, x, xold1, xold2, low, upp, df0, dv, volume_fraction, move=0.2, x_min=1e-3, x_max=1.0,
               tol=1e-13):
    """One MMA update.  Returns (x_new, low, upp, lam): the new design, the
    asymptotes it used (state for the next update) and the multiplier."""
    x = np.asarray(x, dtype=np.float64)
    N = x.size
    dv = np.asarray(dv, dtype=np.float64)
    lo, up = mma_asymptotes(it, x, np.asarray(xold1, float), np.asarray(xold2, float), np.asarray(low, float),
                            np.asarray(upp, float), x_min, x_max)
    span = x_max - x_min
    alpha = np.maximum.reduce([np.full(N, x_min), lo + MMA_ALBEFA * (x - lo), x - move * span])
    beta = np.minimum.reduce([np.full(N, x_max), up - MMA_ALBEFA * (up - x), x + move * span])
    p0, q0 = mma_terms(x, lo, up, np.asarray(df0, dtype=np.float64), x_min, x_max)
    g1 = dv / N
    p1, q1 = mma_terms(x, lo, up, g1, x_min, x_max)
    f1 = float(g1 @ x) - volume_fraction
    r1 = f1 - float(np.sum(p1 / (up - x) + q1 / (x - lo)))

    def x_of(lam):
        P, Q = np.sqrt(p0 + lam * p1), np.sqrt(q0 + lam * q1)
        return np.clip((P * lo + Q * up) / (P + Q), alpha, beta)

    def dual_slope(lam):
        xl = x_of(lam)
        return float(np.sum(p1 / (up - xl) + q1 / (xl - lo))) + r1 - max(0.0, lam - MMA_C)

    if dual_slope(0.0) <= 0.0:
        lam = 0.0
    else:
        a, b = np.log(1e-40), np.log(1e40)
        while b - a > tol:
            m = 0.5 * (a + b)
            if dual_slope(np.exp(m)) > 0.0:
                a = m
            else:
                b = m
        lam = float(np.exp(0.5 * (a + b)))
    return x_of(lam), lo, up, lam


def mma_subproblem_objective(x_new, x, lo, up, df0, dv, volume_fraction, x_min=1e-3, x_max=1.0):
    """The approximate problem's objective and constraint at x_new (for tests)."""
    N = x.size
    p0, q0 = mma_terms(x, lo, up, df0, x_min, x_max)
    p1, q1 = mma_terms(x, lo, up, dv / N, x_min, x_max)
    r1 = float(dv @ x) / N - volume_fraction - float(np.sum(p1 / (up - x) + q1 / (x - lo)))
    f0 = float(np.sum(p0 / (up - x_new) + q0 / (x_new - lo)))
    g1 = float(np.sum(p1 / (up - x_new) + q1 / (x_new - lo))) + r1
    return f0, g1
