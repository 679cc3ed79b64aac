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
