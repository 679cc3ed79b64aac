"""GPU parity of the paper's own state and adjoint pair (section 2.1 eq.
(material) source f0 (1 - rho^p), T_D = 100 on the patch, section 2.3
mean-temperature objective) against the oracle, through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import KMAX, P, field, patch_mask, rel, to_dev  # noqa: E402
from oracle import q1  # noqa: E402

pytestmark = pytest.mark.gpu

TD, F0 = 100.0, 1.0


@pytest.fixture(scope="module")
def pkg():
    import paper_2410_06850_amd as p
    return p


def _oracle_pair(g, rho, mask, kmin, f0):
    td = np.where(mask.astype(bool), TD, 0.0)
    A = q1.assemble(g, q1.conductivity(rho, kmin, KMAX, P))
    f = q1.heat_source_load(g, rho, f0, P)
    T = q1.solve_direct(A, f, mask, td)
    w = q1.mean_temperature_weights(g)
    u = q1.adjoint_solve(A, w, mask)
    return td, f, T, w, u, q1.sensitivity_heat_source(g, rho, T, u, kmin, KMAX, P, f0)


@pytest.mark.parametrize("n,kind,kmin,rho_dtype,H,sd", [
    (16, "noise", 1e-3, torch.float64, 8, 2),
    (16, "grf", 1e-4, torch.float64, 8, 2),
    (12, "grf", 1e-2, torch.float32, 4, 3),
])
def test_paper_pair_matches_oracle(pkg, n, kind, kmin, rho_dtype, H, sd):
    print(f"case paper-pair cube{n}_{kind} kmin={kmin} rho={rho_dtype}", flush=True)
    rho = field(n, kind, 3)
    if rho_dtype == torch.float32:
        rho = rho.astype(np.float32).astype(np.float64)  # the oracle sees the stored values
    mask = patch_mask(n)
    g = q1.Grid(n)
    td, f, T, w, u, dc = _oracle_pair(g, rho, mask, kmin, F0)
    s = pkg.Solver(n, H=H, sd=sd)
    s.setup(to_dev(rho, rho_dtype), kmin, KMAX, P, to_dev(mask, torch.uint8), to_dev(td))
    fg = s.heat_source_load(F0)
    assert rel(fg.cpu().numpy(), f) <= 1e-14
    wg = s.mean_temperature_weights()
    assert rel(wg.cpu().numpy(), w) <= 1e-14
    Tg, info = s.solve(fg, rtol=1e-12, maxit=1000)
    ug, info_u = s.solve_adjoint(wg, rtol=1e-12, maxit=1000)
    dcg = s.sensitivity_heat_source(Tg, ug, F0)
    A = q1.assemble(g, q1.conductivity(rho, kmin, KMAX, P))
    errs = (rel(Tg.cpu().numpy(), T), rel(ug.cpu().numpy(), u), rel(dcg.cpu().numpy(), dc),
            q1.relative_residual(A, Tg.cpu().numpy(), f, mask, td))
    print(f"  it {info.iterations}/{info_u.iterations} err T {errs[0]:.2e} u {errs[1]:.2e} dc {errs[2]:.2e} "
          f"res {errs[3]:.2e}", flush=True)
    assert info.code == 0 and info_u.code == 0
    assert errs[3] <= 1e-12 * (1 + 1e-2)
    # solution bound: rounding times the condition number (~1e5 for the contrast-1e4 field)
    tol = 1e-10 if kind == "noise" else 1e-8
    assert errs[0] <= tol and errs[1] <= tol
    assert errs[2] <= 1e-8
    # f0 = 0 reduces to the stiffness-only sensitivity kernel
    d0 = s.sensitivity_heat_source(Tg, ug, 0.0)
    d1 = s.sensitivity(Tg, ug)
    assert torch.equal(d0, d1)


def test_mean_temperature_autograd_and_fd(pkg):
    """Autograd of the mean temperature: oracle gradient and a central finite
    difference through the GPU solver."""
    print("case mean-temperature autograd cube16_noise", flush=True)
    n, kmin = 16, 1e-3
    rho = field(n, "noise", 4)
    mask = patch_mask(n)
    g = q1.Grid(n)
    td, f, T, w, u, dc = _oracle_pair(g, rho, mask, kmin, F0)
    s = pkg.Solver(n, H=8, sd=2)
    m, tdd = to_dev(mask, torch.uint8), to_dev(td)
    r = to_dev(rho).requires_grad_(True)
    c = pkg.autograd.mean_temperature(r, s, kmin, KMAX, P, m, tdd, f0=F0, rtol=1e-12, maxit=1000)
    assert abs(float(c) - float(w @ T)) <= 1e-10 * abs(float(w @ T))
    c.backward()
    assert rel(r.grad.cpu().numpy(), dc) <= 1e-8
    d = np.random.default_rng(8).uniform(-1, 1, rho.size)
    eps = 1e-5
    vals = []
    for sgn in (1, -1):
        with torch.no_grad():
            vals.append(float(pkg.autograd.mean_temperature(to_dev(rho + sgn * eps * d), s, kmin, KMAX, P, m, tdd,
                                                            f0=F0, rtol=1e-13, maxit=1000)))
    fdv = (vals[0] - vals[1]) / (2 * eps)
    err = abs(fdv - float(r.grad.cpu().numpy() @ d)) / abs(fdv)
    print(f"  FD relative error {err:.2e}")
    assert err <= 1e-5


def test_heat_source_entry_points_reject_bad_input(pkg):
    from paper_2410_06850_amd import _lib as L
    s = pkg.Solver(8, H=4, sd=2)
    f = torch.empty(s.nnodes, dtype=torch.float64, device="cuda")
    # before any set-up: state error, nothing launched
    assert L.lib().msmg_heat_source_load(s._h, 1.0, f.data_ptr(), None) < 0
    assert L.lib().msmg_sensitivity_heat_source(s._h, f.data_ptr(), f.data_ptr(), 1.0, f.data_ptr(), None) < 0
    rho = field(8, "noise", 0)
    s.setup(to_dev(rho), 1e-3, KMAX, P, to_dev(patch_mask(8), torch.uint8))
    with pytest.raises(L.MsmgError):
        s.heat_source_load(float("nan"))
    dc = torch.empty(s.nelem, dtype=torch.float64, device="cuda")
    with pytest.raises(L.MsmgError):
        s.sensitivity_heat_source(f, f, float("inf"), out=dc)
    # the adjoint is required: a NULL lambda is rejected
    assert L.lib().msmg_sensitivity_heat_source(s._h, f.data_ptr(), None, 1.0, dc.data_ptr(), None) < 0


def test_mean_temperature_continuation(pkg):
    """Design-level interpolation on the paper's problem: 8^3 -> 16^3, the
    second level starting from the injected design of the first."""
    print("case continuation cube8->cube16 mean temperature", flush=True)

    def make_mask(n):
        return to_dev(patch_mask(n), torch.uint8)

    def make_fixed(n):
        return to_dev(np.where(patch_mask(n).astype(bool), TD, 0.0))

    x, levels = pkg.topopt.continuation(lambda n: pkg.Solver(n, H=4, sd=2), make_mask, 8, (4, 3), 0.1,
                                        make_fixed=make_fixed, kmin=1e-4, objective="mean_temperature", f0=F0,
                                        maxit=2000)
    assert [lv["n"] for lv in levels] == [8, 16]
    assert x.numel() == 16 ** 3
    for lv in levels:
        obj = [h["objective"] for h in lv["history"]]
        print(f"  n={lv['n']} objective {obj}", flush=True)
        assert all(np.isfinite(obj))
        assert abs(lv["history"][-1]["volume"] - 0.1) <= 1e-6
        assert all(h["adjoint_iterations"] > 0 for h in lv["history"])
    h1 = levels[0]["history"]
    assert h1[-1]["objective"] < h1[0]["objective"]
