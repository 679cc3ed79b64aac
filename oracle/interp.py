"""Oracle, part 3: moving fields between a coarse and a 2x refined mesh.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper (section 3, interpolation technique; section 4.1) optimises at a low
resolution and carries the result to the doubled resolution, without naming
the transfer operator.  The readings used here:
  * temperatures: evaluate the coarse trilinear (Q1) function at the fine
    nodes -- the exact embedding of the coarse Q1 space in the fine one;
  * densities: element injection, each coarse element value copied to its 8
    children (the element-wise constant field is unchanged as a function).
"""
from __future__ import annotations

import numpy as np


def _q1_eval_1d(nc, nf):
    """Fine-node positions along one axis as (left coarse node, weight of right)."""
    t = np.arange(nf + 1) * (nc / nf)          # fine node position in coarse units
    left = np.minimum(np.floor(t).astype(np.int64), nc - 1)
    w = t - left
    return left, w


def prolong_nodal(tc, nc):
    """Coarse nodal field ((nz+1),(ny+1),(nx+1)) -> its values at the 2x-refined nodes."""
    ncx, ncy, ncz = nc
    tc = np.asarray(tc, dtype=np.float64).reshape(ncz + 1, ncy + 1, ncx + 1)
    lx, wx = _q1_eval_1d(ncx, 2 * ncx)
    ly, wy = _q1_eval_1d(ncy, 2 * ncy)
    lz, wz = _q1_eval_1d(ncz, 2 * ncz)
    out = np.zeros((2 * ncz + 1, 2 * ncy + 1, 2 * ncx + 1))
    for az in (0, 1):
        fz = wz if az else 1.0 - wz
        for ay in (0, 1):
            fy = wy if ay else 1.0 - wy
            for ax in (0, 1):
                fx = wx if ax else 1.0 - wx
                vals = tc[np.ix_(lz + az, ly + ay, lx + ax)]
                out += fz[:, None, None] * fy[None, :, None] * fx[None, None, :] * vals
    return out


def inject_element(rc, nc):
    """Coarse element field (nz, ny, nx) -> 2x-refined element field (each value 8 times)."""
    ncx, ncy, ncz = nc
    rc = np.asarray(rc).reshape(ncz, ncy, ncx)
    return np.repeat(np.repeat(np.repeat(rc, 2, axis=0), 2, axis=1), 2, axis=2)
