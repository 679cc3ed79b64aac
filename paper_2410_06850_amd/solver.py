"""Torch-facing wrapper of the C ABI: device memory and streams come from
PyTorch, every step of the computation runs in libmsmg.so.

Layouts: element tensors are (nz, ny, nx) or flat, nodal tensors
(nz+1, ny+1, nx+1) or flat, all C-contiguous on the current HIP device.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name, dtype, numel, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, the solver on {device}")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} entries, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


_DT = {torch.float64: L.MSMG_F64, torch.float32: L.MSMG_F32}


def _info(info):
    d = {}
    for k, _ in L.Info._fields_:
        v = getattr(info, k)
        d[k] = list(v) if isinstance(v, ctypes.Array) else v
    return SolveInfo(d)


class SolveInfo(dict):
    __getattr__ = dict.__getitem__


class Solver:
    """PCG with the three-grid multiscale preconditioner on an nx*ny*nz mesh.

    discretisation="q1" (default): trilinear elements, unknowns on the
    (nx+1)(ny+1)(nz+1) nodes, a nodal Dirichlet mask.  discretisation="tpfa":
    the paper's cell-centred two-point flux finite volumes, unknowns on the
    nx*ny*nz cells, the "mask" of set-up holds each cell's Dirichlet face bits
    and the smoothing interval defaults to [0.2, 2].  ``nnodes`` is the
    number of unknowns either way."""

    def __init__(self, nx, ny=None, nz=None, lx=1.0, ly=1.0, lz=1.0, device=None, discretisation="q1", **options):
        if not torch.cuda.is_available():
            raise RuntimeError("the MsMG solver needs a HIP GPU")
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        if discretisation not in ("q1", "tpfa"):
            raise ValueError("discretisation must be 'q1' or 'tpfa'")
        self.tpfa = discretisation == "tpfa"
        e = 0 if self.tpfa else 1
        self.nnodes = (self.nx + e) * (self.ny + e) * (self.nz + e)
        self.nelem = self.nx * self.ny * self.nz
        self.volume = float(lx) * float(ly) * float(lz)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if self.tpfa:
            options = dict(options, discretisation=L.MSMG_TPFA)
            options.setdefault("cheb_lo", 0.2)
            options.setdefault("cheb_hi", 2.0)
        self.opts = L.default_options(**options)
        self._tune_cache = self.opts.tune_cache  # keep the bytes alive
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(L.lib().msmg_create(ctypes.byref(h), self.nx, self.ny, self.nz, lx, ly, lz, ctypes.byref(self.opts)),
                    "msmg_create")
        self._h = h
        self._keep = []
        self.version = 0  # bumped by every set-up (autograd checks it)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().msmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up ---------------------------------------------------------------
    def setup(self, rho, kmin, kmax, p, mask, fixed_values=None):
        rho = _need(rho, "rho", None, self.nelem, self.device)
        if rho.dtype not in _DT:
            raise TypeError("rho must be float64 or float32")
        mask = _need(mask, "mask", torch.uint8, self.nnodes, self.device)
        fv = None
        if fixed_values is not None:
            fv = _need(fixed_values, "fixed_values", torch.float64, self.nnodes, self.device)
        L.check(L.lib().msmg_setup(self._h, _ptr(rho), _DT[rho.dtype], float(kmin), float(kmax), int(p), _ptr(mask),
                                   _ptr(fv) if fv is not None else None, _stream()), "msmg_setup")
        self.kmin, self.kmax, self.p = float(kmin), float(kmax), int(p)
        self.version += 1
        return self

    # -- solves and products --------------------------------------------------
    def solve(self, f, T=None, rtol=1e-8, maxit=1000, use_x0=False, T_lo=None):
        """Solve A T = f.  With T_lo (a tensor like f) the double-double iterate is
        returned as T + T_lo; otherwise T holds it rounded to binary64."""
        f = _need(f, "f", torch.float64, self.nnodes, self.device)
        if T is None:
            T = torch.empty_like(f)
            use_x0 = False
        else:
            _need(T, "T", torch.float64, self.nnodes, self.device)
        if T_lo is not None:
            _need(T_lo, "T_lo", torch.float64, self.nnodes, self.device)
        info = L.Info()
        code = L.check(L.lib().msmg_solve(self._h, _ptr(f), _ptr(T), _ptr(T_lo) if T_lo is not None else None,
                                          int(bool(use_x0)), float(rtol), int(maxit), ctypes.byref(info), _stream()),
                       "msmg_solve")
        out = _info(info)
        out["code"] = code
        return T, out

    def solve_adjoint(self, g, lam=None, rtol=1e-8, maxit=1000, use_x0=False, lam_lo=None):
        """Adjoint solve A_FF u_F = g_F with zero fixed entries (section 2.3)."""
        g = _need(g, "g", torch.float64, self.nnodes, self.device)
        if lam is None:
            lam = torch.empty_like(g)
            use_x0 = False
        else:
            _need(lam, "lam", torch.float64, self.nnodes, self.device)
        if lam_lo is not None:
            _need(lam_lo, "lam_lo", torch.float64, self.nnodes, self.device)
        info = L.Info()
        code = L.check(L.lib().msmg_solve_adjoint(self._h, _ptr(g), _ptr(lam),
                                                  _ptr(lam_lo) if lam_lo is not None else None, int(bool(use_x0)),
                                                  float(rtol), int(maxit), ctypes.byref(info), _stream()),
                       "msmg_solve_adjoint")
        out = _info(info)
        out["code"] = code
        return lam, out

    def solve_pair(self, f, g, rtol=1e-8, maxit=1000, T=None, lam=None, T_lo=None, lam_lo=None):
        """State solve A T = f and adjoint solve A_FF lambda = g together (one
        set-up, shared coefficient reads); needs Solver(..., pair_rhs=1).
        Returns (T, lambda, info_T, info_lambda)."""
        f = _need(f, "f", torch.float64, self.nnodes, self.device)
        g = _need(g, "g", torch.float64, self.nnodes, self.device)
        T = torch.empty_like(f) if T is None else _need(T, "T", torch.float64, self.nnodes, self.device)
        lam = torch.empty_like(g) if lam is None else _need(lam, "lam", torch.float64, self.nnodes, self.device)
        for t, nm in ((T_lo, "T_lo"), (lam_lo, "lam_lo")):
            if t is not None:
                _need(t, nm, torch.float64, self.nnodes, self.device)
        i1, i2 = L.Info(), L.Info()
        code = L.check(L.lib().msmg_solve_pair(self._h, _ptr(f), _ptr(T), _ptr(T_lo) if T_lo is not None else None,
                                               _ptr(g), _ptr(lam), _ptr(lam_lo) if lam_lo is not None else None,
                                               float(rtol), int(maxit), ctypes.byref(i1), ctypes.byref(i2),
                                               _stream()), "msmg_solve_pair")
        outs = []
        for inf in (i1, i2):
            o = _info(inf)
            o["code"] = code
            outs.append(o)
        return T, lam, outs[0], outs[1]

    def oc_update(self, x, dc, dv, volume_fraction, move=0.2, eta=0.5, x_min=1e-3, out=None):
        """Optimality-criteria update with the volume multiplier found on the GPU;
        returns (x_new, lambda) with lambda a 0-d device tensor."""
        for t, nm in ((x, "x"), (dc, "dc"), (dv, "dv")):
            _need(t, nm, torch.float64, self.nelem, self.device)
        out = torch.empty_like(x) if out is None else _need(out, "out", torch.float64, self.nelem, self.device)
        lam = torch.empty((), dtype=torch.float64, device=self.device)
        L.check(L.lib().msmg_oc_update(self._h, _ptr(x), _ptr(dc), _ptr(dv), float(volume_fraction), float(move),
                                       float(eta), float(x_min), _ptr(out), _ptr(lam), _stream()), "msmg_oc_update")
        return out, lam

    def mma_update(self, it, x, xold1, xold2, low, upp, df0, dv, volume_fraction, move=0.2, x_min=1e-3, out=None):
        """Method of moving asymptotes step (update number `it`); low and upp are
        updated in place; returns (x_new, lambda) with lambda a 0-d device tensor."""
        for t, nm in ((x, "x"), (xold1, "xold1"), (xold2, "xold2"), (low, "low"), (upp, "upp"), (df0, "df0"),
                      (dv, "dv")):
            _need(t, nm, torch.float64, self.nelem, self.device)
        out = torch.empty_like(x) if out is None else _need(out, "out", torch.float64, self.nelem, self.device)
        lam = torch.empty((), dtype=torch.float64, device=self.device)
        L.check(L.lib().msmg_mma_update(self._h, int(it), _ptr(x), _ptr(xold1), _ptr(xold2), _ptr(low), _ptr(upp),
                                        _ptr(df0), _ptr(dv), float(volume_fraction), float(move), float(x_min),
                                        _ptr(out), _ptr(lam), _stream()), "msmg_mma_update")
        return out, lam

    def apply(self, x, y=None):
        x = _need(x, "x", torch.float64, self.nnodes, self.device)
        y = torch.empty_like(x) if y is None else _need(y, "y", torch.float64, self.nnodes, self.device)
        L.check(L.lib().msmg_apply(self._h, _ptr(x), _ptr(y), _stream()), "msmg_apply")
        return y

    def dot(self, a, b):
        """a^T b as a 0-d device tensor (fixed summation order, msmg_dot)."""
        if a.numel() != b.numel():
            raise ValueError("a and b must have the same length")
        _need(a, "a", torch.float64, a.numel(), self.device)
        _need(b, "b", torch.float64, a.numel(), self.device)
        out = torch.empty((), dtype=torch.float64, device=self.device)
        L.check(L.lib().msmg_dot(self._h, _ptr(a), _ptr(b), a.numel(), _ptr(out), _stream()), "msmg_dot")
        return out

    def scale(self, x, c=1.0, s=None, out=None):
        """c * s * x with s a 0-d device tensor (or None), msmg_scale."""
        _need(x, "x", torch.float64, x.numel(), self.device)
        if s is not None:
            s = _need(s.reshape(()).to(torch.float64).contiguous(), "s", torch.float64, 1, self.device)
        out = torch.empty_like(x) if out is None else _need(out, "out", torch.float64, x.numel(), self.device)
        L.check(L.lib().msmg_scale(_ptr(x), x.numel(), float(c), _ptr(s) if s is not None else None, _ptr(out),
                                   _stream()), "msmg_scale")
        return out

    def time_apply(self, x, reps=50):
        """Mean time (ms) of the PCG's operator-apply kernel over reps back-to-back launches on p = x."""
        x = _need(x, "x", torch.float64, self.nnodes, self.device)
        ms = ctypes.c_double()
        L.check(L.lib().msmg_time_apply(self._h, _ptr(x), int(reps), ctypes.byref(ms), _stream()), "msmg_time_apply")
        return ms.value

    def precondition(self, r, z=None):
        r = _need(r, "r", torch.float64, self.nnodes, self.device)
        z = torch.empty_like(r) if z is None else _need(z, "z", torch.float64, self.nnodes, self.device)
        L.check(L.lib().msmg_precondition(self._h, _ptr(r), _ptr(z), _stream()), "msmg_precondition")
        return z

    def sensitivity(self, T, lam=None, out=None):
        T = _need(T, "T", torch.float64, self.nnodes, self.device)
        if lam is not None:
            _need(lam, "lam", torch.float64, self.nnodes, self.device)
        out = (torch.empty(self.nelem, dtype=torch.float64, device=self.device) if out is None
               else _need(out, "out", torch.float64, self.nelem, self.device))
        L.check(L.lib().msmg_sensitivity(self._h, _ptr(T), _ptr(lam) if lam is not None else None, _ptr(out),
                                         _stream()), "msmg_sensitivity")
        return out

    def sensitivity_heat_source(self, T, lam, f0, out=None):
        """dc/drho with the design-dependent source f0 (1 - rho^p) (lam: the adjoint)."""
        T = _need(T, "T", torch.float64, self.nnodes, self.device)
        lam = _need(lam, "lam", torch.float64, self.nnodes, self.device)
        out = (torch.empty(self.nelem, dtype=torch.float64, device=self.device) if out is None
               else _need(out, "out", torch.float64, self.nelem, self.device))
        L.check(L.lib().msmg_sensitivity_heat_source(self._h, _ptr(T), _ptr(lam), float(f0), _ptr(out), _stream()),
                "msmg_sensitivity_heat_source")
        return out

    def heat_source_load(self, f0=1.0):
        """Nodal load of the source f0 (1 - rho^p) for the set-up density."""
        f = torch.empty(self.nnodes, dtype=torch.float64, device=self.device)
        L.check(L.lib().msmg_heat_source_load(self._h, float(f0), _ptr(f), _stream()), "msmg_heat_source_load")
        return f

    def mean_temperature_weights(self):
        """Nodal weights w with w^T T = (1/|Omega|) int T (the mean-temperature objective)."""
        return self.element_load(None, 1.0 / self.volume)

    def element_load(self, src=None, const=1.0):
        f = torch.empty(self.nnodes, dtype=torch.float64, device=self.device)
        if src is not None:
            _need(src, "src", torch.float64, self.nelem, self.device)
        L.check(L.lib().msmg_element_load(self._h, _ptr(src) if src is not None else None, float(const), _ptr(f),
                                          _stream()), "msmg_element_load")
        return f

    def export(self, what, count, dtype=torch.float64):
        out = torch.empty(count, dtype=dtype)
        L.check(L.lib().msmg_export(self._h, int(what), ctypes.c_void_p(out.data_ptr()),
                                    out.numel() * out.element_size()), "msmg_export")
        return out

    def plan(self):
        return L.query_plan(self.nx, self.ny, self.nz, self.opts)


def density_filter(x, n, radius=1.5, transpose=False, out=None):
    """Hat-weight density filter on an (nx,ny,nz) element mesh (or its adjoint)."""
    nx, ny, nz = n
    _need(x, "x", torch.float64, nx * ny * nz, x.device)
    out = torch.empty_like(x) if out is None else _need(out, "out", torch.float64, nx * ny * nz, x.device)
    L.check(L.lib().msmg_density_filter(nx, ny, nz, float(radius), _ptr(x), _ptr(out), int(bool(transpose)),
                                        _stream()), "msmg_density_filter")
    return out


def prolong_nodal(Tc, n):
    """Coarse nodal field on an (nx,ny,nz) mesh -> values at the 2x-refined nodes."""
    nx, ny, nz = n
    _need(Tc, "Tc", torch.float64, (nx + 1) * (ny + 1) * (nz + 1), Tc.device)
    Tf = torch.empty((2 * nz + 1) * (2 * ny + 1) * (2 * nx + 1), dtype=torch.float64, device=Tc.device)
    L.check(L.lib().msmg_prolong_nodal(nx, ny, nz, _ptr(Tc), _ptr(Tf), _stream()), "msmg_prolong_nodal")
    return Tf


def prolong_element(rc, n):
    """Coarse element field -> 2x-refined element field (injection)."""
    nx, ny, nz = n
    if rc.dtype not in (torch.float64, torch.float32, torch.bfloat16):
        raise TypeError("element field must be float64, float32 or bfloat16")
    _need(rc, "rc", None, nx * ny * nz, rc.device)
    dt = {torch.float64: L.MSMG_F64, torch.float32: L.MSMG_F32, torch.bfloat16: L.MSMG_BF16}[rc.dtype]
    rf = torch.empty(8 * nx * ny * nz, dtype=rc.dtype, device=rc.device)
    L.check(L.lib().msmg_prolong_element(nx, ny, nz, _ptr(rc), _ptr(rf), dt, _stream()), "msmg_prolong_element")
    return rf
