"""GPU parity of the fine-level kernels against the oracle (through the C ABI)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import KMAX, P, dev, field, patch_mask, rel, to_dev  # noqa: E402
from oracle import interp, q1  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def msmg():
    import paper_2410_06850_amd as pkg
    return pkg


def _smoother_solver(pkg, n, box=(1.0, 1.0, 1.0), H=8, **kw):
    nx, ny, nz = n
    return pkg.Solver(nx, ny, nz, *box, pc_kind=1, H=H, autotune=0, **kw)


@pytest.mark.parametrize("shape,box,rho_dt", [
    ((16, 16, 16), (1.0, 1.0, 1.0), "f64"),
    ((13, 9, 11), (1.3, 0.9, 1.1), "f64"),
    ((24, 17, 9), (1.0, 1.0, 1.0), "f32"),
    # node counts along x of k * 64 + 1 (the last march tile also computes the
    # final column), k * 64 (exact fit) and k * 64 + 2
    ((64, 12, 10), (1.2, 0.7, 0.9), "f64"),
    ((128, 9, 7), (1.0, 1.0, 1.0), "f64"),
    ((63, 8, 8), (1.0, 1.0, 1.0), "f32"),
    ((65, 6, 9), (1.0, 1.0, 1.0), "f64"),
])
def test_apply_matches_oracle(msmg, shape, box, rho_dt):
    nx, ny, nz = shape
    print(f"case apply {shape} {box} {rho_dt}", flush=True)
    g = q1.Grid(nx, ny, nz, *box)
    rng = np.random.default_rng(1)
    rho = rng.uniform(1e-3, 1.0, g.nelem)
    if rho_dt == "f32":
        rho = rho.astype(np.float32).astype(np.float64)
    mask = (rng.uniform(size=g.nnodes) < 0.05).astype(np.uint8)
    mask[0] = 1
    x = rng.standard_normal(g.nnodes)
    kmin = 1e-4
    A = q1.masked_operator(q1.assemble(g, q1.conductivity(rho, kmin, KMAX, P)), mask)
    want = A @ x
    s = _smoother_solver(msmg, shape, box, H=min(8, min(shape)))
    s.setup(to_dev(rho, torch.float32 if rho_dt == "f32" else torch.float64), kmin, KMAX, P, to_dev(mask, torch.uint8))
    y = s.apply(to_dev(x)).cpu().numpy()
    # rounding bound of a 27-term row in difference form: each product and
    # difference carries a few ulps of the row's absolute terms (|A| |x|)_n
    absrow = abs(A) @ np.abs(x)
    ratio = np.abs(y - want) / absrow
    print(f"  max |y - Ax| / (|A||x|) = {ratio.max():.2e} (eps = 2.2e-16); relative to max|Ax|: "
          f"{np.abs(y - want).max() / np.abs(want).max():.2e}")
    assert np.all(np.abs(y - want) <= 64 * np.finfo(np.float64).eps * absrow)
    assert np.abs(y - want).max() <= 1e-14 * np.abs(want).max()


def test_sensitivity_and_load_match_oracle(msmg):
    n = 12
    print("case sensitivity 12^3", flush=True)
    g = q1.Grid(n)
    rng = np.random.default_rng(2)
    rho = field(n, "noise", 3)
    mask = patch_mask(n)
    T = rng.standard_normal(g.nnodes)
    lam = rng.standard_normal(g.nnodes)
    lam[mask.astype(bool)] = 0.0
    s = _smoother_solver(msmg, (n, n, n), H=4)
    s.setup(to_dev(rho), 1e-3, KMAX, P, to_dev(mask, torch.uint8))
    got = s.sensitivity(to_dev(T), to_dev(lam)).cpu().numpy()
    want = q1.sensitivity(g, rho, T, lam, 1e-3, KMAX, P)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    Tz = T.copy()
    got = s.sensitivity(to_dev(Tz)).cpu().numpy()
    Tfree = np.where(mask.astype(bool), 0.0, Tz)
    want = q1.sensitivity(g, rho, Tz, Tfree, 1e-3, KMAX, P)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    f = s.element_load(const=1.0).cpu().numpy()
    assert np.abs(f - q1.element_load(g, 1.0)).max() <= 1e-17
    src = rng.uniform(size=g.nelem)
    f = s.element_load(src=to_dev(src)).cpu().numpy()
    assert np.abs(f - q1.element_load(g, src)).max() <= 1e-16


def test_interpolation_matches_oracle(msmg):
    nc = (5, 3, 4)
    print("case interpolation", flush=True)
    rng = np.random.default_rng(3)
    tc = rng.standard_normal((nc[2] + 1) * (nc[1] + 1) * (nc[0] + 1))
    tf = msmg.prolong_nodal(to_dev(tc), nc).cpu().numpy()
    assert np.abs(tf - interp.prolong_nodal(tc, nc).ravel()).max() <= 1e-15
    rc = rng.uniform(size=nc[0] * nc[1] * nc[2])
    for dt in (torch.float64, torch.float32):
        rf = msmg.prolong_element(to_dev(rc, dt), nc).cpu().numpy()
        want = interp.inject_element(torch.tensor(rc).to(dt).double().numpy(), nc).ravel()
        assert np.array_equal(rf.astype(np.float64), want)


def test_smoother_pcg_matches_direct_solve(msmg):
    n = 16
    print("case smoother-pcg 16^3", flush=True)
    g = q1.Grid(n)
    rho = field(n, "noise", 0)
    mask = patch_mask(n)
    kmin = 1e-3
    A = q1.assemble(g, q1.conductivity(rho, kmin, KMAX, P))
    f = q1.element_load(g, 1.0)
    Td = q1.solve_direct(A, f, mask)
    s = _smoother_solver(msmg, (n, n, n))
    s.setup(to_dev(rho), kmin, KMAX, P, to_dev(mask, torch.uint8))
    T, info = s.solve(to_dev(f), rtol=1e-12, maxit=5000)
    T = T.cpu().numpy()
    assert info.code == 0, info
    assert q1.relative_residual(A, T, f, mask) <= 1e-12
    assert rel(T, Td) <= 1e-10
    # fixed temperature 100 shifts the solution by 100
    tfix = np.full(g.nnodes, 100.0)
    s.setup(to_dev(rho), kmin, KMAX, P, to_dev(mask, torch.uint8), fixed_values=to_dev(tfix))
    T100, info = s.solve(to_dev(f), rtol=1e-12, maxit=5000)
    assert np.abs(T100.cpu().numpy() - Td - 100.0).max() <= 1e-8


def test_error_paths(msmg):
    import paper_2410_06850_amd._lib as L
    print("case error paths", flush=True)
    n = 8
    s = _smoother_solver(msmg, (n, n, n), H=4)
    f = torch.zeros((n + 1) ** 3, dtype=torch.float64, device=dev())
    with pytest.raises(L.MsmgError) as e:
        s.solve(f)
    assert e.value.code == L.MSMG_ESTATE
    rho = to_dev(field(n))
    with pytest.raises(L.MsmgError) as e:
        s.setup(rho, 0.0, 1.0, 3, to_dev(patch_mask(n), torch.uint8))
    assert e.value.code == L.MSMG_EINVAL
    with pytest.raises(L.MsmgError) as e:
        s.setup(rho, 1e-3, 1.0, 3, torch.zeros((n + 1) ** 3, dtype=torch.uint8, device=dev()))
    assert e.value.code == L.MSMG_ESINGULAR
    with pytest.raises(L.MsmgError) as e:
        msmg.Solver(n, H=16)
    assert e.value.code == L.MSMG_EINVAL
    # zero load: zero solution
    s.setup(rho, 1e-3, 1.0, 3, to_dev(patch_mask(n), torch.uint8))
    T, info = s.solve(f)
    assert info.code == 0 and float(T.abs().max()) == 0.0


@pytest.mark.parametrize("tpfa", [False, True])
def test_time_apply_leaves_the_solver_usable(msmg, tpfa):
    """msmg_time_apply runs the PCG apply kernel on p = x and reports a time;
    x with p^T A p = 0 is refused; a solve afterwards is unchanged."""
    import paper_2410_06850_amd._lib as L
    print(f"case time-apply tpfa={tpfa}", flush=True)
    n = 16
    rho = to_dev(field(n))
    if tpfa:
        import synth
        s = msmg.Solver(n, discretisation="tpfa", H=8, sd=2)
        s.setup(rho, 1e-3, KMAX, P, to_dev(synth.dirichlet_patch_faces(n, n, n).ravel(), torch.uint8))
    else:
        s = msmg.Solver(n, H=8, sd=2)
        s.setup(rho, 1e-3, KMAX, P, to_dev(patch_mask(n), torch.uint8))
    f = s.element_load(const=1.0)
    T0, i0 = s.solve(f, rtol=1e-10)
    ms = s.time_apply(T0, 5)
    assert ms > 0.0
    with pytest.raises(L.MsmgError) as e:
        s.time_apply(torch.zeros_like(f), 2)
    assert e.value.code == L.MSMG_EINVAL
    T1, i1 = s.solve(f, rtol=1e-10)
    assert i1.iterations == i0.iterations and torch.equal(T0, T1)


def test_dot_and_scale(msmg):
    """msmg_dot against an exact (fsum) dot product, reproducible bit for bit;
    msmg_scale is c * s * x with s read on the device."""
    import math
    print("case dot/scale", flush=True)
    n = 16
    s = msmg.Solver(n, H=8, sd=2)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((2, s.nnodes))
    da, db = to_dev(a), to_dev(b)
    d1, d2 = s.dot(da, db), s.dot(da, db)
    exact = math.fsum(a * b)
    assert abs(float(d1) - exact) <= 1e-13 * math.fsum(np.abs(a * b))
    assert torch.equal(d1, d2)
    g = torch.tensor(0.75, dtype=torch.float64, device=dev())
    y = s.scale(da, 2.0, g).cpu().numpy()
    assert np.array_equal(y, (2.0 * 0.75) * a)
    assert np.array_equal(s.scale(da, 3.0).cpu().numpy(), 3.0 * a)
