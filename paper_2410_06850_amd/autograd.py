"""Differentiable solve and compliance (section 2.3: the state system and the
adjoint system share the matrix and, here, the preconditioner set-up).

``solve(rho, f, solver, ...)`` returns T with A(rho) T = f (fixed values from
the set-up).  Its backward runs the adjoint solve A_FF u_F = (dL/dT)_F with the
same set-up, then the element sensitivity kernel:
    dL/drho_e = -u_e^T (dA/drho_e) T_e,   dL/df = u (zero on fixed nodes).
``compliance(rho, f, solver, ...)`` returns c = f^T T; with zero fixed values
its adjoint is T itself, so the backward needs no second solve.
``mean_temperature(rho, solver, ...)`` is the paper's own pair: the source
f0 (1 - rho^p) of eq. (material), fixed values T_D, and the mean temperature
c = (1/|Omega|) int T of eq. (cost function).  Its backward solves the adjoint
A_FF u_F = w_F (w: the mean weights) and adds the df/drho term:
    dc/drho_e = u^T (df/drho_e - dA/drho_e T).
The objective values and the chain-rule scalings by the upstream gradient run
in the library too (msmg_dot, msmg_scale); this module only wires the calls.
"""
from __future__ import annotations

import torch


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, f, solver, kmin, kmax, p, mask, fixed_values, rtol, maxit):
        solver.setup(rho.detach().contiguous(), kmin, kmax, p, mask, fixed_values)
        T, info = solver.solve(f.detach().contiguous(), rtol=rtol, maxit=maxit)
        if info.code != 0:
            raise RuntimeError(f"state solve did not converge: {dict(info)}")
        ctx.solver, ctx.version, ctx.rtol, ctx.maxit = solver, solver.version, rtol, maxit
        ctx.save_for_backward(T)
        solver.last_info = info
        return T

    @staticmethod
    def backward(ctx, gT):
        solver = ctx.solver
        if solver.version != ctx.version:
            raise RuntimeError("the solver was set up again before backward; the adjoint needs the forward set-up")
        (T,) = ctx.saved_tensors
        u, info = solver.solve_adjoint(gT.detach().contiguous(), rtol=ctx.rtol, maxit=ctx.maxit)
        if info.code != 0:
            raise RuntimeError(f"adjoint solve did not converge: {dict(info)}")
        g_rho = solver.sensitivity(T, u) if ctx.needs_input_grad[0] else None
        g_f = u if ctx.needs_input_grad[1] else None
        return g_rho, g_f, None, None, None, None, None, None, None, None


class _Compliance(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, f, solver, kmin, kmax, p, mask, rtol, maxit):
        solver.setup(rho.detach().contiguous(), kmin, kmax, p, mask, None)
        T, info = solver.solve(f.detach().contiguous(), rtol=rtol, maxit=maxit)
        if info.code != 0:
            raise RuntimeError(f"state solve did not converge: {dict(info)}")
        ctx.solver, ctx.version = solver, solver.version
        ctx.save_for_backward(T)
        solver.last_info = info
        return solver.dot(f.detach().contiguous(), T)

    @staticmethod
    def backward(ctx, gc):
        solver = ctx.solver
        if solver.version != ctx.version:
            raise RuntimeError("the solver was set up again before backward; the adjoint needs the forward set-up")
        (T,) = ctx.saved_tensors
        # zero fixed values: the adjoint of c = f^T T is u = T
        g_rho = solver.scale(solver.sensitivity(T), 1.0, gc) if ctx.needs_input_grad[0] else None
        g_f = solver.scale(T, 2.0, gc) if ctx.needs_input_grad[1] else None  # c = f^T A^-1 f
        return g_rho, g_f, None, None, None, None, None, None, None


class _MeanTemperature(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, solver, kmin, kmax, p, mask, fixed_values, f0, rtol, maxit):
        solver.setup(rho.detach().contiguous(), kmin, kmax, p, mask, fixed_values)
        f = solver.heat_source_load(f0)
        T, info = solver.solve(f, rtol=rtol, maxit=maxit)
        if info.code != 0:
            raise RuntimeError(f"state solve did not converge: {dict(info)}")
        w = solver.mean_temperature_weights()
        ctx.solver, ctx.version, ctx.f0, ctx.rtol, ctx.maxit = solver, solver.version, f0, rtol, maxit
        ctx.save_for_backward(T, w)
        solver.last_info = info
        return solver.dot(w, T)

    @staticmethod
    def backward(ctx, gc):
        solver = ctx.solver
        if solver.version != ctx.version:
            raise RuntimeError("the solver was set up again before backward; the adjoint needs the forward set-up")
        T, w = ctx.saved_tensors
        u, info = solver.solve_adjoint(w, rtol=ctx.rtol, maxit=ctx.maxit)
        if info.code != 0:
            raise RuntimeError(f"adjoint solve did not converge: {dict(info)}")
        solver.last_adjoint_info = info
        g_rho = solver.scale(solver.sensitivity_heat_source(T, u, ctx.f0), 1.0, gc)
        return g_rho, None, None, None, None, None, None, None, None, None


def solve(rho, f, solver, kmin, kmax, p, mask, fixed_values=None, rtol=1e-8, maxit=1000):
    """T = A(rho)^-1 f (differentiable in rho and f)."""
    return _Solve.apply(rho, f, solver, kmin, kmax, p, mask, fixed_values, rtol, maxit)


def compliance(rho, f, solver, kmin, kmax, p, mask, rtol=1e-8, maxit=1000):
    """c = f^T T with T = A(rho)^-1 f and zero fixed values (differentiable)."""
    return _Compliance.apply(rho, f, solver, kmin, kmax, p, mask, rtol, maxit)


def mean_temperature(rho, solver, kmin, kmax, p, mask, fixed_values=None, f0=1.0, rtol=1e-8, maxit=1000):
    """c = (1/|Omega|) int T with A(rho) T = f(rho), f from the source f0 (1 - rho^p)
    and the given fixed values (differentiable in rho)."""
    return _MeanTemperature.apply(rho, solver, kmin, kmax, p, mask, fixed_values, f0, rtol, maxit)
