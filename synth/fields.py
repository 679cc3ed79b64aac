"""Seeded design fields and the Dirichlet mask of the model problem.

Layouts: element arrays are (nz, ny, nx) C-order (x fastest), nodal arrays are
(nz+1, ny+1, nx+1) C-order.  Nothing here evaluates the discretisation or the
solver; the functions only draw or shape input data.

Model problem (paper, section 2.1 and its domain figure): unit cube, fixed
temperature on a centred square patch of the bottom face (z = 0), adiabatic
elsewhere.  The paper leaves the design fields of its experiments to its own
optimiser runs, which are not available; thresholded Gaussian random fields
with the paper's resolutions and contrasts stand in for them.
"""
from __future__ import annotations

import hashlib

import numpy as np
import scipy.fft


def uniform_noise_rho(n, seed=0, base=0.3, amp=0.05, shape=None):
    """Near-uniform density: ``base + U(-amp, amp)`` per element, float64."""
    shape = (n, n, n) if shape is None else tuple(shape)
    rng = np.random.default_rng(seed)
    return base + rng.uniform(-amp, amp, shape)


def grf_raw(n, ell, seed=0, dtype=np.float64, shape=None):
    """Unthresholded Gaussian random field with covariance exp(-r^2 / (2 ell^2)).

    White noise is filtered, axis by axis and periodically, with a Gaussian of
    standard deviation ``ell / sqrt(2)`` elements (the convolution of two such
    Gaussians has variance ``ell^2``).
    """
    shape = (n, n, n) if shape is None else tuple(shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape, dtype=dtype)
    s = float(ell) / np.sqrt(2.0)
    for axis in range(3):
        m = shape[axis]
        freq = np.fft.rfftfreq(m)  # cycles per element
        tf = np.exp(-0.5 * (2.0 * np.pi * freq * s) ** 2).astype(dtype)
        bshape = [1, 1, 1]
        bshape[axis] = -1
        spec = scipy.fft.rfft(w, axis=axis, workers=-1)
        spec *= tf.reshape(bshape)
        w = scipy.fft.irfft(spec, n=m, axis=axis, workers=-1).astype(dtype, copy=False)
        del spec
    return w


def threshold_field(w, vf=0.4, lo=1e-3, hi=1.0, dtype=np.float64):
    """Binary field: the largest ``vf`` fraction of ``w`` becomes ``hi``, the rest ``lo``.

    The cut is the exact order statistic of index floor((1 - vf) * size).
    """
    flat = w.reshape(-1)
    idx = int(np.floor((1.0 - vf) * flat.size))
    idx = min(max(idx, 0), flat.size - 1)
    thr = np.partition(flat, idx)[idx]
    out = np.where(w >= thr, hi, lo).astype(dtype)
    return out


def grf_rho(n, ell, seed=0, vf=0.4, lo=1e-3, hi=1.0, dtype=np.float64, shape=None):
    """Thresholded GRF density with volume fraction ``vf`` of ``hi`` material."""
    raw_dtype = np.float32 if dtype == np.float32 else np.float64
    w = grf_raw(n, ell, seed, dtype=raw_dtype, shape=shape)
    return threshold_field(w, vf=vf, lo=lo, hi=hi, dtype=dtype)


def block_average(w, f=2):
    """Average over f^3 blocks (used to derive a coarser companion field)."""
    nz, ny, nx = w.shape
    return w.reshape(nz // f, f, ny // f, f, nx // f, f).mean(axis=(1, 3, 5))


def dirichlet_patch_mask(nx, ny, nz, frac=(1, 5)):
    """Nodal mask (uint8, 1 = fixed temperature) of the centred bottom patch.

    A node (i, j, 0) is fixed when |x - 1/2| <= f/2 and |y - 1/2| <= f/2 with
    f = num/den, i.e. ``den * |2 i - nx| <= num * nx`` (integer exact).
    """
    num, den = frac
    mask = np.zeros((nz + 1, ny + 1, nx + 1), dtype=np.uint8)
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    inx = den * np.abs(2 * i - nx) <= num * nx
    iny = den * np.abs(2 * j - ny) <= num * ny
    mask[0] = (iny[:, None] & inx[None, :]).astype(np.uint8)
    return mask


def dirichlet_patch_faces(nx, ny, nz, frac=(1, 5)):
    """Cell face flags (uint8 per cell, (nz, ny, nx)) of the same centred bottom
    patch for cell-centred unknowns: bit 4 (the -z face) is set on the bottom
    cells whose face centre lies in the patch, ``den * |2 i + 1 - nx| <= num * nx``
    and the same along y.  Bits 0..5 name the -x, +x, -y, +y, -z, +z faces.
    """
    num, den = frac
    flags = np.zeros((nz, ny, nx), dtype=np.uint8)
    i = np.arange(nx)
    j = np.arange(ny)
    inx = den * np.abs(2 * i + 1 - nx) <= num * nx
    iny = den * np.abs(2 * j + 1 - ny) <= num * ny
    flags[0] = np.where(iny[:, None] & inx[None, :], np.uint8(1 << 4), np.uint8(0))
    return flags


def field_sha256(a):
    """SHA-256 of the raw bytes of a C-contiguous array."""
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
