"""Topology-optimisation loop around the solver (the experiments of section 4
minimise a thermal objective over densities with a gradient-based update;
here: compliance c = f^T T, a hat density filter and an optimality-criteria
update with a volume constraint, all on the GPU).

Each iteration: rho_phys = H(x); c = f^T A(rho_phys)^-1 f (set-up rebuilt for
rho_phys, PCG solve); dc/dx = H^T dc/drho_phys (autograd: sensitivity kernel,
then the filter's adjoint); x <- OC(x, dc/dx, H^T 1).
"""
from __future__ import annotations

import time

import torch

from . import autograd
from .solver import density_filter


class DensityFilter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, n, radius):
        ctx.n, ctx.radius = n, radius
        return density_filter(x.detach().contiguous(), n, radius)

    @staticmethod
    def backward(ctx, g):
        return density_filter(g.detach().contiguous(), ctx.n, ctx.radius, transpose=True), None, None


def optimize(solver, mask, iterations=20, volume_fraction=0.3, x0=0.3, radius=1.5, move=0.2, eta=0.5,
             kmin=1e-6, kmax=1.0, p=3, rtol=1e-8, maxit=1000, x_min=1e-3, log=None):
    """Run `iterations` design updates; returns (x, history)."""
    n = (solver.nx, solver.ny, solver.nz)
    dev = solver.device
    f = solver.element_load(const=1.0)
    x = torch.full((solver.nelem,), float(x0), dtype=torch.float64, device=dev)
    ones = torch.ones_like(x)
    dv = density_filter(ones, n, radius, transpose=True)
    hist = []
    for it in range(iterations):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xv = x.clone().requires_grad_(True)
        rho = DensityFilter.apply(xv, n, radius)
        c = autograd.compliance(rho, f, solver, kmin, kmax, p, mask, rtol=rtol, maxit=maxit)
        c.backward()
        info = solver.last_info
        x_new, lam = solver.oc_update(x, xv.grad, dv, volume_fraction, move=move, eta=eta, x_min=x_min)
        change = float((x_new - x).abs().max())
        x = x_new
        torch.cuda.synchronize()
        rec = dict(iteration=it, compliance=float(c), change=change, volume=float(x.mean()),
                   pcg_iterations=info["iterations"], setup_ms=info["setup_ms"], solve_ms=info["solve_ms"],
                   step_s=time.perf_counter() - t0, lam=float(lam))
        hist.append(rec)
        if log:
            log(rec)
    return x, hist
