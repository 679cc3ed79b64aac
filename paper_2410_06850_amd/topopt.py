"""Topology-optimisation loop around the solver (the experiments of section 4
minimise a thermal objective over densities with a gradient-based update;
here a hat density filter and a moving-asymptotes (MMA) or optimality-criteria
update with a volume constraint, all on the GPU).

Objectives: compliance c = f^T T (fixed unit source, zero fixed values), or
the paper's mean temperature (source f0 (1 - rho^p) of eq. (material), fixed
values T_D, eq. (cost function)).

Each iteration: rho_phys = H(x); c(rho_phys) (set-up rebuilt for rho_phys,
PCG solve); dc/dx = H^T dc/drho_phys (autograd: adjoint solve where needed,
sensitivity kernel, then the filter's adjoint); x <- OC(x, dc/dx, H^T 1), or
the method of moving asymptotes (section 2.3's optimiser) with the volume
constraint H^T 1 . x / N <= volume fraction.

``continuation`` is the interpolation technique of section 4 at the design
level: optimise on a coarse mesh, inject the design into the 2x mesh
(`prolong_element`) and continue there.
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
             kmin=1e-6, kmax=1.0, p=3, rtol=1e-8, maxit=1000, x_min=1e-3, log=None,
             objective="compliance", fixed_values=None, f0=1.0, optimizer="oc"):
    """Run `iterations` design updates; returns (x, history).  x0: a constant or
    an element tensor (the initial design); objective: "compliance" or
    "mean_temperature" (with fixed_values and the source amplitude f0);
    optimizer: "oc" (optimality criteria) or "mma" (the method of moving
    asymptotes of section 2.3, on the objective scaled by its first value and
    the volume constraint dv . x / N <= volume_fraction)."""
    if optimizer not in ("oc", "mma"):
        raise ValueError(f"unknown optimizer {optimizer}")
    n = (solver.nx, solver.ny, solver.nz)
    dev = solver.device
    if objective not in ("compliance", "mean_temperature"):
        raise ValueError(f"unknown objective {objective}")
    f = solver.element_load(const=1.0) if objective == "compliance" else None
    if torch.is_tensor(x0):
        if x0.numel() != solver.nelem:
            raise ValueError("x0 must have one value per element")
        x = x0.detach().to(device=dev, dtype=torch.float64).reshape(-1).clone()
    else:
        x = torch.full((solver.nelem,), float(x0), dtype=torch.float64, device=dev)
    ones = torch.ones_like(x)
    dv = density_filter(ones, n, radius, transpose=True)
    hist = []
    if optimizer == "mma":
        # MMA state: the last two designs and the asymptotes
        xold1, xold2 = x.clone(), x.clone()
        low, upp = torch.zeros_like(x), torch.ones_like(x)
        c_scale = None
    for it in range(iterations):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xv = x.clone().requires_grad_(True)
        rho = DensityFilter.apply(xv, n, radius)
        if objective == "compliance":
            c = autograd.compliance(rho, f, solver, kmin, kmax, p, mask, rtol=rtol, maxit=maxit)
        else:
            c = autograd.mean_temperature(rho, solver, kmin, kmax, p, mask, fixed_values, f0=f0, rtol=rtol,
                                          maxit=maxit)
        c.backward()
        info = solver.last_info
        if optimizer == "oc":
            x_new, lam = solver.oc_update(x, xv.grad, dv, volume_fraction, move=move, eta=eta, x_min=x_min)
        else:
            if c_scale is None:
                c_scale = 1.0 / max(abs(float(c.detach())), 1e-300)
            x_new, lam = solver.mma_update(it, x, xold1, xold2, low, upp, xv.grad * c_scale, dv, volume_fraction,
                                           move=move, x_min=x_min)
            xold2, xold1 = xold1, x
        change = float((x_new - x).abs().max())
        x = x_new
        torch.cuda.synchronize()
        rec = dict(iteration=it, objective=float(c.detach()), change=change, volume=float(x.mean()),
                   volume_physical=float(torch.dot(dv, x)) / solver.nelem, optimizer=optimizer,
                   pcg_iterations=info["iterations"], setup_ms=info["setup_ms"], solve_ms=info["solve_ms"],
                   adjoint_iterations=(solver.last_adjoint_info["iterations"] if objective != "compliance" else 0),
                   step_s=time.perf_counter() - t0, lam=float(lam))
        hist.append(rec)
        if log:
            log(rec)
    return x, hist


def continuation(make_solver, make_mask, n0, schedule, volume_fraction, x0=None, make_fixed=None, log=None, **kw):
    """Design-level interpolation: `schedule` lists the iterations per level on
    meshes n0, 2 n0, 4 n0, ...; the final design of a level, injected into the
    2x mesh, starts the next.  make_solver(n), make_mask(n) and make_fixed(n)
    (optional) give each level's solver, fixed-node mask and fixed values; the
    other keywords go to `optimize`.  Returns (x of the last level, per-level
    records with the history)."""
    from .solver import prolong_element

    n = int(n0)
    x = volume_fraction if x0 is None else x0
    levels = []
    for li, its in enumerate(schedule):
        if li > 0:
            x = prolong_element(x, (n // 2, n // 2, n // 2))
        solver = make_solver(n)
        fixed = make_fixed(n) if make_fixed else None
        t0 = time.perf_counter()
        x, hist = optimize(solver, make_mask(n), iterations=its, volume_fraction=volume_fraction, x0=x,
                           fixed_values=fixed, log=(lambda r, n=n: log(dict(r, n=n))) if log else None, **kw)
        torch.cuda.synchronize()
        levels.append(dict(n=n, iterations=its, seconds=time.perf_counter() - t0, history=hist))
        solver.close()
        del solver
        n *= 2
    return x, levels
