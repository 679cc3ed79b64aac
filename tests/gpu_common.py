"""Shared helpers of the GPU parity tests (inputs from synth, references from oracle)."""
import numpy as np
import torch

import synth
from oracle import msmg as omsmg
from oracle import q1

KMAX, P = 1.0, 3


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to(dev()).contiguous().reshape(-1)


def field(n, kind="noise", seed=0, ell=4):
    if kind == "noise":
        return synth.uniform_noise_rho(n, seed).ravel()
    return synth.grf_rho(n, ell, seed=seed).ravel()


def patch_mask(n):
    return synth.dirichlet_patch_mask(n, n, n).ravel()


def oracle_hier(n, rho, kmin, mask, H, sd, Lc=4, Lcc=17, deg=2):
    g = q1.Grid(n)
    return g, omsmg.Hierarchy(g, rho, kmin, KMAX, P, mask, omsmg.Options(H=H, sd=sd, Lc=Lc, Lcc=Lcc, cheb_degree=deg))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_sin_angle(Pa, Pb, m):
    """Largest principal angle sine between span(Pa) and span(Pb) in the m-weighted inner product."""
    qa, _ = np.linalg.qr(np.sqrt(m)[:, None] * Pa)
    qb, _ = np.linalg.qr(np.sqrt(m)[:, None] * Pb)
    s = np.linalg.svd(qa.T @ qb, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))
