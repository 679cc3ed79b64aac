"""Pins of the oracle's Q1 discretisation (CPU only).

Each test checks the oracle against something other than itself: Gauss
quadrature of the trilinear shape functions, closed-form solutions,
invariants of the Neumann operator, and finite differences.
"""
import numpy as np
import pytest

import synth
from oracle import q1


def _gauss_element(hx, hy, hz, what):
    """Brute-force element matrices by 2-point Gauss quadrature of Q1 shape functions."""
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)
    pts = (g + 1.0) / 2.0  # on [0, 1]
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for xi in pts:
        for eta in pts:
            for zeta in pts:
                w = 0.125 * hx * hy * hz  # each weight 1/2 per axis on [0,1], times volume
                N = np.zeros(8)
                dN = np.zeros((8, 3))
                for a in range(8):
                    ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
                    fx = xi if ax else 1 - xi
                    fy = eta if ay else 1 - eta
                    fz = zeta if az else 1 - zeta
                    sx = 1.0 if ax else -1.0
                    sy = 1.0 if ay else -1.0
                    sz = 1.0 if az else -1.0
                    N[a] = fx * fy * fz
                    dN[a] = [sx * fy * fz / hx, fx * sy * fz / hy, fx * fy * sz / hz]
                K += w * dN @ dN.T
                M += w * np.outer(N, N)
    return K if what == "K" else M


@pytest.mark.parametrize("h", [(1.0, 1.0, 1.0), (0.25, 0.5, 0.125), (0.1, 0.3, 0.7)])
def test_element_matrices_match_quadrature(h):
    assert np.allclose(q1.element_stiffness(*h), _gauss_element(*h, "K"), rtol=0, atol=1e-14 * max(h) / min(h) ** 2)
    assert np.allclose(q1.element_mass(*h), _gauss_element(*h, "M"), rtol=0, atol=1e-15)


def test_unit_cube_element_closed_form():
    K = q1.element_stiffness(1.0, 1.0, 1.0)
    for a in range(8):
        for b in range(8):
            ndiff = bin(a ^ b).count("1")
            want = {0: 1.0 / 3.0, 1: 0.0, 2: -1.0 / 12.0, 3: -1.0 / 12.0}[ndiff]
            assert abs(K[a, b] - want) <= 1e-16
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-15)
    assert abs(np.linalg.eigvalsh(K).max() - 0.5) < 1e-14
    # K0 = h * Khat for cubes of side h
    assert np.allclose(q1.element_stiffness(0.25, 0.25, 0.25), 0.25 * K, atol=1e-16)


def test_conductivity_law():
    rho = np.array([0.0, 0.5, 1.0, 1e-3])
    k = q1.conductivity(rho, 1e-6, 1.0, 3)
    assert np.allclose(k, 1e-6 + rho ** 3 * (1.0 - 1e-6), rtol=1e-15)
    assert k[0] == 1e-6 and k[2] == 1.0


def test_neumann_operator_invariants():
    rng = np.random.default_rng(3)
    g = q1.Grid(5, 4, 6)
    k = 10.0 ** rng.uniform(-6, 0, g.nelem)
    A = q1.assemble(g, k)
    assert np.abs(A @ np.ones(g.nnodes)).max() <= 1e-14 * np.abs(A).max() * 27
    x, y = rng.standard_normal((2, g.nnodes))
    assert abs(x @ (A @ y) - y @ (A @ x)) <= 1e-13 * np.abs(x @ (A @ y)) + 1e-300
    assert x @ (A @ x) >= 0
    # 21-point pattern for cubes: axis neighbours have coefficient exactly 0
    g2 = q1.Grid(4)
    A2 = q1.assemble(g2, np.ones(g2.nelem)).tocsr()
    n = g2.node_index(2, 2, 2)
    row = A2.getrow(n)
    nz = {int(c) for c, v in zip(row.indices, row.data) if v != 0.0}
    assert len(nz) == 21
    for d in (1, g2.nnx, g2.nnx * g2.nny):
        assert A2[n, n + d] == 0.0 and A2[n, n - d] == 0.0


def _layered_exact(zn, kz):
    """T(z) = int_0^z (1 - s) / k(s) ds for piecewise-constant k per layer."""
    T = np.zeros(len(zn))
    for i in range(1, len(zn)):
        a, b = zn[i - 1], zn[i]
        T[i] = T[i - 1] + ((b - a) - 0.5 * (b * b - a * a)) / kz[i - 1]
    return T


@pytest.mark.parametrize("contrast", [1.0, 1e3, 1e6])
def test_layered_exact_solution(contrast):
    n = 6
    g = q1.Grid(n)
    rng = np.random.default_rng(7)
    kz = np.where(rng.uniform(size=n) < 0.5, 1.0, 1.0 / contrast)
    k = np.repeat(kz, n * n)  # element layers along z
    A = q1.assemble(g, k)
    mask = np.zeros((n + 1,) * 3, dtype=np.uint8)
    mask[0] = 1
    f = q1.element_load(g, 1.0)
    T = q1.solve_direct(A, f, mask.ravel())
    zn = np.arange(n + 1) / n
    want = _layered_exact(zn, kz)
    T3 = T.reshape(n + 1, n + 1, n + 1)
    tol = 1e-12 if contrast == 1.0 else 1e-15 * contrast * 100
    for kk in range(n + 1):
        assert np.abs(T3[kk] - want[kk]).max() <= tol * max(1.0, abs(want).max())


def test_manufactured_solution_second_order():
    errs = []
    for n in (4, 8, 16):
        g = q1.Grid(n)
        ix, jy, kz = g.node_coords()
        x, y, z = ix / n, jy / n, kz / n
        u = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
        src = 3 * np.pi ** 2 * u
        f = q1.assemble_mass(g) @ src
        A = q1.assemble(g, np.ones(g.nelem))
        mask = ((ix == 0) | (ix == n) | (jy == 0) | (jy == n) | (kz == 0) | (kz == n)).astype(np.uint8)
        T = q1.solve_direct(A, f, mask)
        errs.append(np.abs(T - u).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.7 <= r2 <= 4.3, errs
    assert r1 > 3.0


def test_dirichlet_value_shift():
    """Fixed temperature T_D shifts the solution by T_D (A 1 = 0, adiabatic elsewhere)."""
    n = 6
    g = q1.Grid(n)
    rho = synth.uniform_noise_rho(n, 1).ravel()
    k = q1.conductivity(rho, 1e-3, 1.0, 3)
    A = q1.assemble(g, k)
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    f = q1.element_load(g, 1.0)
    T0 = q1.solve_direct(A, f, mask)
    T100 = q1.solve_direct(A, f, mask, np.full(g.nnodes, 100.0))
    assert np.abs(T100 - T0 - 100.0).max() < 1e-10


def test_load_and_energy_identity():
    n = 8
    g = q1.Grid(n)
    f = q1.element_load(g, 1.0)
    assert abs(f.sum() - 1.0) < 1e-14  # integral of the unit source over the unit cube
    rho = synth.uniform_noise_rho(n, 0).ravel()
    k = q1.conductivity(rho, 1e-3, 1.0, 3)
    A = q1.assemble(g, k)
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    T = q1.solve_direct(A, f, mask)
    c = q1.compliance(f, T)
    assert abs(c - T @ (A @ T)) <= 1e-12 * c
    assert q1.relative_residual(A, T, f, mask) < 1e-12


def _compliance_of(g, rho, mask, kmin, kmax, p):
    k = q1.conductivity(rho, kmin, kmax, p)
    A = q1.assemble(g, k)
    f = q1.element_load(g, 1.0)
    T = q1.solve_direct(A, f, mask)
    return q1.compliance(f, T), T, A, f


def test_sensitivity_identities_and_fd():
    n = 6
    g = q1.Grid(n)
    kmin, kmax, p = 1e-3, 1.0, 3
    rho = synth.uniform_noise_rho(n, 2).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    c, T, A, f = _compliance_of(g, rho, mask, kmin, kmax, p)
    lam = q1.adjoint_solve(A, f, mask)
    assert np.abs(lam - T).max() <= 1e-12 * np.abs(T).max()   # compliance is self-adjoint
    dc = q1.sensitivity(g, rho, T, T, kmin, kmax, p)
    assert (dc <= 0).all()
    # Euler identity: sum_e rho_e dc_e = -p (c - k_min T^T A0 T)
    A0 = q1.assemble(g, np.ones(g.nelem))
    lhs = rho @ dc
    rhs = -p * (c - kmin * T @ (A0 @ T))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)
    # central finite difference along a random direction
    d = np.random.default_rng(5).standard_normal(g.nelem)
    eps = 1e-6
    cp = _compliance_of(g, rho + eps * d, mask, kmin, kmax, p)[0]
    cm = _compliance_of(g, rho - eps * d, mask, kmin, kmax, p)[0]
    fd = (cp - cm) / (2 * eps)
    assert abs(fd - dc @ d) <= 1e-6 * abs(dc @ d)


def test_general_adjoint_fd():
    """A non-self-adjoint objective L = w^T T: dL/drho from the adjoint matches FD."""
    n = 5
    g = q1.Grid(n)
    kmin, kmax, p = 1e-2, 1.0, 3
    rho = synth.uniform_noise_rho(n, 4).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    w = np.random.default_rng(9).standard_normal(g.nnodes)

    def L(r):
        _, T, A, f = _compliance_of(g, r, mask, kmin, kmax, p)
        return w @ T, T, A

    L0, T, A = L(rho)
    lam = q1.adjoint_solve(A, w, mask)
    dL = q1.sensitivity(g, rho, T, lam, kmin, kmax, p)
    d = np.random.default_rng(6).standard_normal(g.nelem)
    eps = 1e-6
    fd = (L(rho + eps * d)[0] - L(rho - eps * d)[0]) / (2 * eps)
    assert abs(fd - dL @ d) <= 1e-6 * abs(dL @ d)


def test_heat_source_load_invariants():
    """eq. (material), second line: the design-dependent source and its load."""
    g = q1.Grid(4, 3, 5)
    rho = np.random.default_rng(3).uniform(0.0, 1.0, g.nelem)
    f0, p = 2.5, 3
    fs = q1.heat_source_load(g, rho, f0, p)
    # total heat is the integral of f0 (1 - rho^p) over the box
    assert abs(fs.sum() - f0 * np.sum(1.0 - rho ** 3) * g.vol) <= 1e-14 * abs(fs.sum())
    # void generates f0 everywhere, solid nothing
    assert np.allclose(q1.heat_source_load(g, np.zeros(g.nelem), f0, p), q1.element_load(g, f0), rtol=0, atol=1e-16)
    assert np.abs(q1.heat_source_load(g, np.ones(g.nelem), f0, p)).max() == 0.0
    # p = 1 at rho = 1/2: half the void source
    assert np.allclose(q1.heat_source_load(g, np.full(g.nelem, 0.5), f0, 1), q1.element_load(g, f0 / 2), rtol=1e-15)
    # a single hot element loads exactly its 8 nodes with V/8 each
    r1 = np.ones(g.nelem)
    r1[g.element_index(1, 2, 3)] = 0.0
    f1 = q1.heat_source_load(g, r1, f0, p)
    assert np.count_nonzero(f1) == 8 and np.allclose(f1[f1 != 0], f0 * g.vol / 8)


def test_mean_temperature_weights():
    """eq. (cost function): w^T T is the mean of the Q1 field over the box."""
    g = q1.Grid(6, 4, 5, 2.0, 1.0, 0.5)
    w = q1.mean_temperature_weights(g)
    assert abs(w.sum() - 1.0) < 1e-14
    ix, jy, kz = g.node_coords()
    x, y, z = ix * g.hx, jy * g.hy, kz * g.hz
    # trilinear fields are exact in Q1: mean of x y z over [0,2]x[0,1]x[0,.5] is 1 * 1/2 * 1/4
    assert abs(w @ (x * y * z).ravel() - 0.125) < 1e-14
    # x^2 is integrated by the Q1 interpolant, i.e. the trapezoid rule: (L^2/3 + h^2/6)
    hx = 2.0 / 6
    assert abs(w @ (x ** 2).ravel() - (4.0 / 3 + hx ** 2 / 6)) < 1e-13


def _mean_temperature_of(g, rho, mask, kmin, kmax, p, f0, td):
    A = q1.assemble(g, q1.conductivity(rho, kmin, kmax, p))
    f = q1.heat_source_load(g, rho, f0, p)
    T = q1.solve_direct(A, f, mask, td)
    return q1.mean_temperature_weights(g) @ T, T, A


@pytest.mark.parametrize("kmin,kmax,f0", [(1e-2, 1.0, 1.0), (0.3, 0.3, 1.0), (1e-2, 1.0, 0.0)])
def test_paper_state_adjoint_fd(kmin, kmax, f0):
    """Section 2.3 with the paper's pair: source f0 (1 - rho^p), T_D = 100 on the
    patch, mean-temperature objective.  The adjoint gradient matches central
    finite differences; the three cases pin the full gradient, the source term
    alone (k independent of rho) and the stiffness term alone (f0 = 0: no
    source, so the fixed values vary along the patch, 100 + 50 x, to keep T
    non-constant)."""
    n, p = 5, 3
    g = q1.Grid(n)
    rho = np.random.default_rng(11).uniform(0.2, 0.9, g.nelem)
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    ix = g.node_coords()[0]
    td = np.where(mask != 0, 100.0 + (50.0 * ix * g.hx if f0 == 0.0 else 0.0), 0.0)
    c, T, A = _mean_temperature_of(g, rho, mask, kmin, kmax, p, f0, td)
    lam = q1.adjoint_solve(A, q1.mean_temperature_weights(g), mask)
    assert np.abs(lam[mask != 0]).max() == 0.0
    dc = q1.sensitivity_heat_source(g, rho, T, lam, kmin, kmax, p, f0)
    d = np.random.default_rng(12).standard_normal(g.nelem)
    eps = 1e-6
    fd = (_mean_temperature_of(g, rho + eps * d, mask, kmin, kmax, p, f0, td)[0]
          - _mean_temperature_of(g, rho - eps * d, mask, kmin, kmax, p, f0, td)[0]) / (2 * eps)
    assert abs(fd - dc @ d) <= 1e-6 * abs(dc @ d)
    if f0 == 0.0:
        assert np.array_equal(dc, q1.sensitivity(g, rho, T, lam, kmin, kmax, p))
    if kmin == kmax:
        assert np.abs(q1.sensitivity(g, rho, T, lam, kmin, kmax, p)).max() == 0.0


def test_elementwise_apply_matches_assembly():
    rng = np.random.default_rng(11)
    g = q1.Grid(7, 5, 9, 1.0, 0.5, 2.0)
    k = 10.0 ** rng.uniform(-4, 0, g.nelem)
    x = rng.standard_normal(g.nnodes)
    mask = (rng.uniform(size=g.nnodes) < 0.1).astype(np.uint8)
    A = q1.assemble(g, k)
    y1 = q1.apply_elementwise(g, k, x, zslab=3)
    assert np.abs(y1 - A @ x).max() <= 1e-13 * np.abs(A @ x).max()
    y2 = q1.apply_elementwise(g, k, x, mask=mask, zslab=4)
    Am = q1.masked_operator(A, mask)
    assert np.abs(y2 - Am @ x).max() <= 1e-13 * np.abs(Am @ x).max()


def test_difference_form_operator():
    """DiffOperator is the masked operator; its rounding does not grow with |x|."""
    rng = np.random.default_rng(12)
    g = q1.Grid(6, 5, 7)
    k = 10.0 ** rng.uniform(-6, 0, g.nelem)
    A = q1.assemble(g, k)
    mask = (rng.uniform(size=g.nnodes) < 0.1).astype(np.uint8)
    D = q1.DiffOperator(A, mask)
    Am = q1.masked_operator(A, mask)
    x = rng.standard_normal(g.nnodes)
    assert np.abs(D @ x - Am @ x).max() <= 1e-13 * np.abs(Am @ x).max()
    # a large shift c on the free nodes leaves rows away from fixed nodes
    # unchanged; x on a 2^-20 grid and c = 2^26 keep x + c exact in binary64
    x = np.round(x * 2.0 ** 20) / 2.0 ** 20
    c = 2.0 ** 26
    fr = ~mask.astype(bool)
    xs = np.where(fr, x + c, 0.0)
    inner = fr & (np.abs(A) @ mask.astype(float) == 0)
    ref = (D @ x)[inner]
    err_diff = np.abs((D @ xs)[inner] - ref).max()
    err_plain = np.abs((Am @ xs)[inner] - ref).max()
    assert err_diff <= 1e-14 * np.abs(ref).max()
    assert err_plain > 1e3 * max(err_diff, 1e-300)
    # residual helpers agree on well-scaled data, with and without a low part
    f = q1.element_load(g, 1.0)
    T = q1.solve_direct(A, f, mask)
    assert abs(q1.relative_residual_diff(A, T, f, mask) - q1.relative_residual(A, T, f, mask)) <= 1e-10
    lo = 1e-20 * rng.standard_normal(g.nnodes)
    assert abs(q1.relative_residual_diff(A, T, f, mask, T_lo=lo) - q1.relative_residual_diff(A, T, f, mask)) <= 1e-10


def test_residual_rows_match_assembled_operator():
    """Node-by-node residual rows (used where the grid is too large to assemble)
    equal f - A T with the scattered sparse matrix, on an uneven box with
    random densities, temperatures and loads; corner, edge, face and interior
    nodes all appear."""
    g = q1.Grid(6, 5, 4, lx=0.6, ly=1.0, lz=0.8)
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.0, 1.0, g.nelem)
    T = rng.standard_normal(g.nnodes)
    T_lo = 1e-17 * rng.standard_normal(g.nnodes)
    f = rng.standard_normal(g.nnodes)
    kmin, kmax, p = 1e-3, 1.0, 3
    A = q1.assemble(g, q1.conductivity(rho, kmin, kmax, p))
    want = f - A @ (T + T_lo)
    nodes = np.arange(g.nnodes)
    got, absum = q1.residual_rows(g, rho, kmin, kmax, p, T, f[nodes], nodes, T_lo=T_lo)
    assert np.all(np.abs(got - want) <= 1e-13 * (absum + np.abs(f)))
    # a float32 density array gives the same rows as its exact float64 upcast
    r32 = rho.astype(np.float32)
    a, _ = q1.residual_rows(g, r32, kmin, kmax, p, T, f[nodes[::7]], nodes[::7])
    b, _ = q1.residual_rows(g, r32.astype(np.float64), kmin, kmax, p, T, f[nodes[::7]], nodes[::7])
    assert np.array_equal(a, b)


def test_element_load_rows_match_full_load():
    g = q1.Grid(5, 4, 3, lx=1.0, ly=0.5, lz=2.0)
    nodes = np.arange(g.nnodes)
    assert np.allclose(q1.element_load_rows(g, 2.5, nodes), q1.element_load(g, 2.5), rtol=1e-15, atol=0)


def test_relative_residual_slabs_matches_assembled():
    """The slab-wise element residual equals the assembled difference-form
    residual (zero fixed values), for several slab heights."""
    g = q1.Grid(7, 6, 5)
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.0, 1.0, g.nelem)
    T = rng.standard_normal(g.nnodes)
    T_lo = 1e-17 * rng.standard_normal(g.nnodes)
    mask = synth.dirichlet_patch_mask(7, 6, 5).ravel()
    T[mask.astype(bool)] = 0.0
    T_lo[mask.astype(bool)] = 0.0
    f = q1.element_load(g, 1.0) + 0.1 * rng.standard_normal(g.nnodes)
    A = q1.assemble(g, q1.conductivity(rho, 1e-4, 1.0, 3))
    want = q1.relative_residual_diff(A, T, f, mask, T_lo=T_lo)
    for zs in (1, 2, 8):
        got = q1.relative_residual_slabs(g, rho, 1e-4, 1.0, 3, T, f, mask, T_lo=T_lo, zslab=zs)
        assert abs(got - want) <= 1e-13 * want
