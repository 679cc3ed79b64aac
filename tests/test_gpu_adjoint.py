"""GPU parity of the adjoint solve, the differentiable solve/compliance and the
design-update kernels (filter, OC) against the oracle (through the C ABI)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import KMAX, P, field, patch_mask, rel, to_dev  # noqa: E402
from oracle import q1, topopt  # noqa: E402

pytestmark = pytest.mark.gpu

N, KMIN = 16, 1e-3


@pytest.fixture(scope="module")
def pkg():
    import paper_2410_06850_amd as p
    return p


@pytest.fixture(scope="module")
def case(pkg):
    rho = field(N, "noise", 0)
    mask = patch_mask(N)
    g = q1.Grid(N)
    s = pkg.Solver(N, H=8, sd=2)
    return g, s, rho, mask


def test_adjoint_solve_ignores_fixed_values(pkg, case):
    print("case adjoint-solve cube16_noise", flush=True)
    g, s, rho, mask = case
    td = np.where(mask.astype(bool), 100.0, 0.0)
    s.setup(to_dev(rho), KMIN, KMAX, P, to_dev(mask, torch.uint8), to_dev(td))
    A = q1.assemble(g, q1.conductivity(rho, KMIN, KMAX, P))
    w = np.random.default_rng(5).standard_normal(g.nnodes)
    lam, info = s.solve_adjoint(to_dev(w), rtol=1e-12, maxit=500)
    assert info.code == 0
    want = q1.adjoint_solve(A, w, mask)
    assert rel(lam.cpu().numpy(), want) <= 1e-10
    assert np.all(lam.cpu().numpy()[mask.astype(bool)] == 0.0)
    # the state solve still sees the fixed values
    f = q1.element_load(g, 1.0)
    T, info = s.solve(to_dev(f), rtol=1e-12, maxit=500)
    assert rel(T.cpu().numpy(), q1.solve_direct(A, f, mask, td)) <= 1e-10


def test_solve_gradient_matches_oracle_and_fd(pkg, case):
    """L = w^T T(rho): autograd gradient vs oracle adjoint sensitivity and a
    central finite difference along a random direction."""
    print("case autograd-solve cube16_noise", flush=True)
    g, s, rho, mask = case
    f = q1.element_load(g, 1.0)
    w = np.random.default_rng(6).standard_normal(g.nnodes)
    r = to_dev(rho).requires_grad_(True)
    fd = to_dev(f).requires_grad_(True)
    T = pkg.autograd.solve(r, fd, s, KMIN, KMAX, P, to_dev(mask, torch.uint8), rtol=1e-12, maxit=500)
    L = torch.dot(to_dev(w), T)
    L.backward()
    A = q1.assemble(g, q1.conductivity(rho, KMIN, KMAX, P))
    To = q1.solve_direct(A, f, mask)
    u = q1.adjoint_solve(A, w, mask)
    want = q1.sensitivity(g, rho, To, u, KMIN, KMAX, P)
    assert rel(r.grad.cpu().numpy(), want) <= 1e-8
    assert rel(fd.grad.cpu().numpy(), u) <= 1e-10
    # finite difference with the GPU solver
    d = np.random.default_rng(7).uniform(-1, 1, rho.size)
    eps = 1e-4
    vals = []
    for sgn in (1, -1):
        with torch.no_grad():
            Tp = pkg.autograd.solve(to_dev(rho + sgn * eps * d), to_dev(f), s, KMIN, KMAX, P,
                                    to_dev(mask, torch.uint8), rtol=1e-12, maxit=500)
        vals.append(float(torch.dot(to_dev(w), Tp)))
    fdv = (vals[0] - vals[1]) / (2 * eps)
    err = abs(fdv - float(r.grad.cpu().numpy() @ d)) / abs(fdv)
    print(f"  FD relative error {err:.2e}")
    assert err <= 1e-5


def test_compliance_gradient_uses_T_as_adjoint(pkg, case):
    print("case autograd-compliance cube16_noise", flush=True)
    g, s, rho, mask = case
    f = q1.element_load(g, 1.0)
    r = to_dev(rho).requires_grad_(True)
    c = pkg.autograd.compliance(r, to_dev(f), s, KMIN, KMAX, P, to_dev(mask, torch.uint8), rtol=1e-12, maxit=500)
    c.backward()
    A = q1.assemble(g, q1.conductivity(rho, KMIN, KMAX, P))
    To = q1.solve_direct(A, f, mask)
    assert abs(float(c.detach()) - q1.compliance(f, To)) <= 1e-10 * abs(q1.compliance(f, To))
    want = q1.sensitivity(g, rho, To, To, KMIN, KMAX, P)
    assert rel(r.grad.cpu().numpy(), want) <= 1e-8
    # the explicit adjoint solve with g = f returns T
    lam, _ = s.solve_adjoint(to_dev(f), rtol=1e-12, maxit=500)
    T, _ = s.solve(to_dev(f), rtol=1e-12, maxit=500)
    assert rel(lam.cpu().numpy(), T.cpu().numpy()) <= 1e-11
    # setting up again before backward is refused
    r2 = to_dev(rho).requires_grad_(True)
    c2 = pkg.autograd.compliance(r2, to_dev(f), s, KMIN, KMAX, P, to_dev(mask, torch.uint8))
    s.setup(to_dev(rho), KMIN, KMAX, P, to_dev(mask, torch.uint8))
    with pytest.raises(RuntimeError):
        c2.backward()


@pytest.mark.parametrize("n,r", [((9, 7, 5), 1.5), ((16, 16, 16), 1.5), ((12, 10, 8), 2.5)])
def test_density_filter_matches_oracle(pkg, n, r):
    print(f"case filter {n} r={r}", flush=True)
    ne = n[0] * n[1] * n[2]
    x = np.random.default_rng(8).random(ne)
    for tr in (False, True):
        got = pkg.density_filter(to_dev(x), n, r, transpose=tr).cpu().numpy()
        assert rel(got, topopt.density_filter(x, n, r, transpose=tr)) <= 1e-14


def test_oc_update_matches_oracle(pkg, case):
    print("case oc-update cube16", flush=True)
    g, s, rho, mask = case
    rng = np.random.default_rng(9)
    x = rng.uniform(0.2, 0.5, g.nelem)
    dc = -rng.uniform(0.1, 5.0, g.nelem)
    dv = rng.uniform(0.5, 1.5, g.nelem)
    xn, lam = s.oc_update(to_dev(x), to_dev(dc), to_dev(dv), 0.3, move=0.2, eta=0.5, x_min=1e-3)
    want, lam_o = topopt.oc_update(x, dc, dv, 0.3, move=0.2, eta=0.5, x_min=1e-3)
    assert abs(float(lam) - lam_o) <= 1e-8 * lam_o
    assert rel(xn.cpu().numpy(), want) <= 1e-8
    assert abs(float(xn.sum()) - 0.3 * g.nelem) <= 1e-6 * g.nelem


@pytest.mark.parametrize("it,shift", [(0, -0.05), (1, -0.02), (4, -0.05), (5, None), (6, -0.3)])
def test_mma_update_matches_oracle(pkg, case, it, shift):
    """MMA step (section 2.3's optimiser) against the oracle: asymptotes (first
    updates and the sign rule), the multiplier of the dual (1e-8) and the new
    design (1e-9), with the volume target just below the design (active
    constraint, lam ~ 2-5), far above a thin design (vf = 1: inactive, lam = 0)
    and far below (unreachable within the move limits: elastic, lam > c).
    The objective gradient is scaled like the loop's (objective / its first
    value, so ~1/N per element)."""
    print(f"case mma-update cube16 it={it} shift={shift}", flush=True)
    g, s, rho, mask = case
    rng = np.random.default_rng(10 + it)
    ne = g.nelem
    x = rng.uniform(0.05, 0.15, ne) if shift is None else rng.uniform(0.2, 0.8, ne)
    x1 = np.clip(x + rng.uniform(-0.05, 0.05, ne), 1e-3, 1.0)
    x2 = np.clip(x1 + rng.uniform(-0.05, 0.05, ne), 1e-3, 1.0)
    low, upp = x - rng.uniform(0.05, 0.5, ne), x + rng.uniform(0.05, 0.5, ne)
    dc = -np.exp(rng.standard_normal(ne)) / ne
    dv = rng.uniform(0.5, 1.5, ne)
    vf = 1.0 if shift is None else float(dv @ x) / ne + shift
    want, lo_o, up_o, lam_o = topopt.mma_update(it, x, x1, x2, low, upp, dc, dv, vf, move=0.2, x_min=1e-3)
    lo_g, up_g = to_dev(low), to_dev(upp)
    xn, lam = s.mma_update(it, to_dev(x), to_dev(x1), to_dev(x2), lo_g, up_g, to_dev(dc), to_dev(dv), vf,
                           move=0.2, x_min=1e-3)
    assert rel(lo_g.cpu().numpy(), lo_o) <= 1e-15 and rel(up_g.cpu().numpy(), up_o) <= 1e-15
    print(f"  lambda gpu {float(lam):.12e} oracle {lam_o:.12e}")
    if shift is None:
        assert lam_o == 0.0 and float(lam) == 0.0
    elif shift == -0.3:
        assert lam_o > 1000.0
    else:
        assert 0.0 < lam_o < 1000.0
    if lam_o != 0.0:
        assert abs(float(lam) - lam_o) <= 1e-8 * lam_o
    assert rel(xn.cpu().numpy(), want) <= 1e-9


def test_topopt_loop_runs_and_decreases_compliance(pkg):
    print("case topopt-loop cube16", flush=True)
    s = pkg.Solver(16, H=8, sd=2)
    x, hist = pkg.topopt.optimize(s, to_dev(patch_mask(16), torch.uint8), iterations=6, kmin=1e-6)
    cs = [h["objective"] for h in hist]
    assert all(np.isfinite(cs))
    assert cs[-1] < cs[0]
    assert abs(hist[-1]["volume"] - 0.3) <= 1e-6


def test_topopt_loop_with_mma(pkg):
    """The loop with the method of moving asymptotes: the compliance falls and
    the physical (filtered) volume meets the constraint."""
    print("case topopt-loop mma cube16", flush=True)
    s = pkg.Solver(16, H=8, sd=2)
    x, hist = pkg.topopt.optimize(s, to_dev(patch_mask(16), torch.uint8), iterations=8, kmin=1e-6, x0=0.3,
                                  optimizer="mma")
    cs = [h["objective"] for h in hist]
    print("  compliance " + " ".join(f"{c:.4g}" for c in cs))
    assert all(np.isfinite(cs)) and cs[-1] < 0.8 * cs[0]
    assert hist[-1]["volume_physical"] <= 0.3 + 1e-6
    assert float(x.min()) >= 1e-3 and float(x.max()) <= 1.0


def test_compliance_gradient_fd_cube32(pkg):
    """The optimisation workload's gradient check: compliance c = f^T T on a
    32^3 instance (near-uniform density, default hierarchy H 8, sd 8), autograd
    gradient against the oracle's adjoint sensitivity (1e-8) and against a
    central finite difference with FP64 perturbations of 1e-6 along a random
    direction (1e-6; section 2.3)."""
    n = 32
    print("case autograd-compliance FD cube32_noise, delta 1e-6", flush=True)
    g = q1.Grid(n)
    rho = field(n, "noise", 4)
    mask = patch_mask(n)
    f = q1.element_load(g, 1.0)
    s = pkg.Solver(n, H=8, sd=8)
    m = to_dev(mask, torch.uint8)
    r = to_dev(rho).requires_grad_(True)
    c = pkg.autograd.compliance(r, to_dev(f), s, KMIN, KMAX, P, m, rtol=1e-12, maxit=500)
    c.backward()
    grad = r.grad.cpu().numpy()
    A = q1.assemble(g, q1.conductivity(rho, KMIN, KMAX, P))
    To = q1.solve_direct(A, f, mask)
    want = q1.sensitivity(g, rho, To, To, KMIN, KMAX, P)
    e_or = rel(grad, want)
    d = np.random.default_rng(8).uniform(-1, 1, rho.size)
    delta = 1e-6
    vals = []
    for sgn in (1, -1):
        with torch.no_grad():
            cv = pkg.autograd.compliance(to_dev(rho + sgn * delta * d), to_dev(f), s, KMIN, KMAX, P, m,
                                         rtol=1e-12, maxit=500)
        vals.append(float(cv))
    fdv = (vals[0] - vals[1]) / (2 * delta)
    e_fd = abs(fdv - float(grad @ d)) / abs(fdv)
    print(f"  oracle gradient rel.err {e_or:.2e}, FD relative error {e_fd:.2e}")
    assert e_or <= 1e-8
    assert e_fd <= 1e-6
