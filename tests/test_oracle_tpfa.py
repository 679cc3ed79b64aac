"""Pins of the oracle's TPFA discretisation and its three-grid hierarchy (CPU only).

Pins: exactness for layered media along each axis (harmonic face means and
the half-cell Dirichlet distance reproduce the exact 1-D solution at the cell
centres), second-order convergence on a manufactured solution with a
non-cubic mesh (face weights |F|/h_d and the load f |K| per axis), the
Neumann kernel and symmetry of the assembled matrix, the closed-form local
spectrum at constant conductivity, the normalisation R_c M R_c^T = I, the
explicit three-grid error-propagation formula, and PCG against direct
solves.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import msmg, q1, tpfa


def _layer_field(grid, axis, kl):
    ex, ey, ez = grid.element_coords()
    return np.asarray(kl)[(ex, ey, ez)[axis]]


def _faces_on(grid, axis, side):
    ex, ey, ez = grid.element_coords()
    c = (ex, ey, ez)[axis]
    n = (grid.nx, grid.ny, grid.nz)[axis]
    bit = 2 * axis + (1 if side > 0 else 0)
    on = (c == 0) if side < 0 else (c == n - 1)
    return np.where(on, 1 << bit, 0).astype(np.uint8)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_layered_medium_is_exact(axis):
    """-(k T')' = 0 across layers, T = a and b on the two end faces: the exact
    solution sampled at the cell centres, to rounding."""
    n = (7, 5, 6)
    grid = q1.Grid(*n, lx=2.0, ly=0.5, lz=0.3)
    rng = np.random.default_rng(axis)
    kl = 10.0 ** rng.uniform(-4, 0, size=n[axis])
    k = _layer_field(grid, axis, kl)
    a, b = 3.0, -1.5
    flags = _faces_on(grid, axis, -1) | _faces_on(grid, axis, +1)
    td = np.where(_faces_on(grid, axis, -1) > 0, a, b)
    t = tpfa.solve_direct(grid, k, flags, np.zeros(grid.nelem), td)
    h = (grid.hx, grid.hy, grid.hz)[axis]
    # resistances in series: half cells at the ends, (h/2)(1/k_i + 1/k_i+1) between centres
    steps = np.concatenate([[0.5 * h / kl[0]], 0.5 * h * (1.0 / kl[:-1] + 1.0 / kl[1:])])
    J = (a - b) / (steps.sum() + 0.5 * h / kl[-1])
    want_layers = a - J * np.cumsum(steps)
    want = _layer_field(grid, axis, want_layers)
    assert np.abs(t - want).max() <= 1e-12 * max(abs(a), abs(b))


def _mms(nx, ny, nz, lx=1.0, ly=2.0, lz=0.5):
    grid = q1.Grid(nx, ny, nz, lx=lx, ly=ly, lz=lz)
    ex, ey, ez = grid.element_coords()
    x, y, z = (ex + 0.5) * grid.hx, (ey + 0.5) * grid.hy, (ez + 0.5) * grid.hz
    ax, ay, az = np.pi / lx, np.pi / ly, np.pi / (2 * lz)

    def kap(x, y, z):
        return 1.0 + 0.5 * (x / lx) * (y / ly) * (z / lz)

    def T(x, y, z):
        return np.cos(ax * x) * np.cos(ay * y) * (2.0 + np.sin(az * z))

    # f = -div(k grad T) at the cell centres, from the closed forms
    k = kap(x, y, z)
    kx = 0.5 * (1 / lx) * (y / ly) * (z / lz)
    ky = 0.5 * (x / lx) * (1 / ly) * (z / lz)
    kz = 0.5 * (x / lx) * (y / ly) * (1 / lz)
    cx, sx = np.cos(ax * x), np.sin(ax * x)
    cy, sy = np.cos(ay * y), np.sin(ay * y)
    gz, dgz, d2gz = 2.0 + np.sin(az * z), az * np.cos(az * z), -az ** 2 * np.sin(az * z)
    Tx, Ty, Tz = -ax * sx * cy * gz, -ay * cx * sy * gz, cx * cy * dgz
    lap = -ax ** 2 * cx * cy * gz - ay ** 2 * cx * cy * gz + cx * cy * d2gz
    f = -(k * lap + kx * Tx + ky * Ty + kz * Tz)
    # Dirichlet on the bottom face (its centre values), zero normal flux elsewhere
    flags = _faces_on(grid, 2, -1)
    td = T(x, y, 0.0)
    t = tpfa.solve_direct(grid, k, flags, tpfa.cell_load(grid, f), td)
    return np.abs(t - T(x, y, z)).max()


def test_manufactured_solution_second_order():
    e1 = _mms(6, 6, 6)
    e2 = _mms(12, 12, 12)
    e3 = _mms(24, 24, 24)
    assert e2 < e1 and e3 < e2
    assert np.log2(e2 / e3) >= 1.8, (e1, e2, e3)


def test_matrix_symmetric_with_neumann_kernel():
    grid = q1.Grid(5, 4, 3, lx=1.0, ly=0.7, lz=1.3)
    k = q1.conductivity(synth.uniform_noise_rho(5, 1, shape=(3, 4, 5)).ravel(), 1e-3, 1.0, 3)
    A = tpfa.assemble(grid, k).toarray()
    assert np.array_equal(A, A.T)
    assert np.abs(A @ np.ones(grid.nelem)).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() >= -1e-12 * np.abs(A).max()
    flags = synth.dirichlet_patch_faces(5, 4, 3, frac=(1, 2)).ravel()
    assert flags.any()
    Ad = tpfa.assemble(grid, k, flags).toarray()
    assert np.linalg.eigvalsh(Ad).min() > 0
    x = np.random.default_rng(0).standard_normal(grid.nelem)
    op = tpfa.Operator(grid, k, flags)
    assert np.abs(op @ x - Ad @ x).max() <= 1e-13 * np.abs(Ad @ x).max()
    with pytest.raises(ValueError):
        bad = np.zeros(grid.nelem, dtype=np.uint8)
        bad[grid.element_index(2, 1, 1)] = 1   # a -x face inside the mesh
        tpfa.check_face_flags(grid, bad)


def _tpfa_closed_form(nx, ny, nz, hx, hy, hz):
    """Eigenvalues of the constant-k Neumann TPFA form against k |K|."""
    def lam(j, n, h):
        return (4.0 / h ** 2) * np.sin(np.pi * j / (2 * n)) ** 2

    a = np.arange(nx)[:, None, None]
    b = np.arange(ny)[None, :, None]
    c = np.arange(nz)[None, None, :]
    return np.sort((lam(a, nx, hx) + lam(b, ny, hy) + lam(c, nz, hz)).ravel())


def _setup(n, H, sd, Lc=4, Lcc=17, rho=None, kmin=1e-3, seed=0, flags=None, deg=2, shape=None):
    shape = shape or (n, n, n)
    g = q1.Grid(shape[2], shape[1], shape[0])
    rho = synth.uniform_noise_rho(n, seed, shape=shape).ravel() if rho is None else rho
    flags = synth.dirichlet_patch_faces(shape[2], shape[1], shape[0]).ravel() if flags is None else flags
    h = tpfa.Hierarchy(g, rho, kmin, 1.0, 3, flags, tpfa.default_options(H=H, sd=sd, Lc=Lc, Lcc=Lcc, cheb_degree=deg))
    return g, h


@pytest.mark.parametrize("rhoval", [1.0, 0.5])
def test_local_eigenpairs_constant_k_closed_form(rhoval):
    n = 20   # runs of 8 and 12 cells
    g, h = _setup(n, 8, 2, Lc=8, rho=np.full(n ** 3, rhoval))
    kval = q1.conductivity(np.array([rhoval]), 1e-3, 1.0, 3)[0]
    for ci, (cx, cy, cz) in enumerate(h.cells):
        (sx, ex), (sy, ey), (sz, ez) = h.runs[0][cx], h.runs[1][cy], h.runs[2][cz]
        want = _tpfa_closed_form(ex - sx, ey - sy, ez - sz, g.hx, g.hy, g.hz)[:8]
        got = h.cell_evals[ci]
        assert abs(got[0]) <= 1e-10 * want[-1]
        assert np.allclose(got[1:], want[1:], rtol=1e-11, atol=0), (ci, got, want)
        nodes, phi = h.cell_basis[ci]
        # eigenvalue 0 belongs to the constant, normalised in the k |K| form
        c0 = np.full(len(nodes), 1.0 / np.sqrt(kval * g.vol * len(nodes)))
        assert np.allclose(phi[:, 0], c0, rtol=1e-9)


def test_local_basis_normalisation_and_partition():
    n = 16
    g, h = _setup(n, 4, 2, kmin=1e-6, rho=synth.grf_rho(n, 4, seed=1).ravel())
    owner = np.full(g.nelem, -1)
    for ci in range(len(h.cells)):
        nodes, phi = h.cell_basis[ci]
        m = h.cell_mass[ci]
        assert np.allclose(m, h.k[nodes] * g.vol)
        G = phi.T @ (m[:, None] * phi)
        assert np.allclose(G, np.eye(phi.shape[1]), atol=1e-12)
        assert (owner[nodes] == -1).all()
        owner[nodes] = ci
    assert (owner >= 0).all()


def test_cc_level_constant_in_kernel():
    n = 16
    g, h = _setup(n, 4, 2, rho=np.full(n ** 3, 1.0))
    for lam in h.cc_evals:
        assert abs(lam[0]) <= 1e-9 * max(1.0, abs(lam[-1]))
    Rcc = h.Rcc.toarray()
    assert np.allclose(Rcc @ Rcc.T, np.eye(h.n_cc), atol=1e-12)
    # the cc stiffness keeps exactly the faces inside one cc cell: a face
    # between cells 7 and 8 along x (coarse cells 1 and 2, cc groups 0 and 1)
    K = h.cc_stiffness()
    a, b = g.element_index(7, 3, 3), g.element_index(8, 3, 3)
    assert K[a, b] == 0.0
    a2, b2 = g.element_index(6, 3, 3), g.element_index(7, 3, 3)
    assert K[a2, b2] < 0.0


def test_three_grid_error_propagation_formula():
    """I - M^-1 A = (I - S^-T A)(I - R_c^T B_c R_c A)(I - S^-1 A) on the TPFA matrices."""
    g, h = _setup(6, 2, 2, Lc=4, Lcc=17)
    nf = g.nelem
    A = h.A_csr.toarray()
    lam, V = sla.eigh(A, np.diag(h.diag))
    o = h.o
    theta, delta = 0.5 * (o.cheb_hi + o.cheb_lo), 0.5 * (o.cheb_hi - o.cheb_lo)

    def cheb_T(d, x):
        x = np.asarray(x, dtype=np.float64)
        return np.where(np.abs(x) <= 1, np.cos(d * np.arccos(np.clip(x, -1, 1))),
                        np.sign(x) ** d * np.cosh(d * np.arccosh(np.maximum(np.abs(x), 1))))

    err = cheb_T(o.cheb_degree, (theta - lam) / delta) / cheb_T(o.cheb_degree, theta / delta)
    Sinv = V @ np.diag((1.0 - err) / lam) @ V.T
    Rc = h.Rc.toarray()
    Ac = h.Ac.toarray()
    blk = np.empty(h.n_c, dtype=np.int64)
    for ci, rows in enumerate(h.cell_rows):
        blk[rows] = ci
    col = np.array([h.colour(*h.cells[b]) for b in blk])
    keep = (blk[:, None] == blk[None, :]) | (col[None, :] < col[:, None])
    Sc = np.where(keep, Ac, 0.0)
    Rcc = h.Rcc.toarray()
    I_c = np.eye(h.n_c)
    Ec = (I_c - np.linalg.solve(Sc.T, Ac)) @ (I_c - Rcc.T @ np.linalg.solve(h.Acc, Rcc @ Ac)) @ \
        (I_c - np.linalg.solve(Sc, Ac))
    Bc = (I_c - Ec) @ np.linalg.inv(Ac)
    I_f = np.eye(nf)
    E = (I_f - Sinv @ A) @ (I_f - Rc.T @ Bc @ Rc @ A) @ (I_f - Sinv @ A)
    Minv_formula = (I_f - E) @ np.linalg.inv(A)
    Minv = np.column_stack([h.precondition(np.eye(nf)[:, j]) for j in range(nf)])
    assert np.abs(Minv - Minv_formula).max() <= 1e-10 * np.abs(Minv).max()
    assert np.abs(Minv - Minv.T).max() <= 1e-10 * np.abs(Minv).max()


@pytest.mark.parametrize("n,H,sd", [(8, 2, 2), (8, 4, 1), (16, 8, 2), (16, 4, 2), (12, 4, 8), (20, 8, 1)])
def test_pcg_matches_direct_solve(n, H, sd):
    g = q1.Grid(n)
    rho = synth.grf_rho(n, 4, seed=n).ravel()
    flags = synth.dirichlet_patch_faces(n, n, n).ravel()
    f = tpfa.cell_load(g, tpfa_source(rho))
    t, res, h = tpfa.solve(g, rho, f, flags, 1e-3, 1.0, 3, tpfa.default_options(H=H, sd=sd), rtol=1e-12, td=100.0)
    assert res.status == "converged" and res.rel_res <= 1e-12
    td = tpfa.solve_direct(g, h.k, flags, f, 100.0)
    assert np.linalg.norm(t - td) / np.linalg.norm(td) <= 1e-10
    assert res.iterations <= 60


def test_smoother_interval_and_positive_preconditioner():
    """D^-1 A of TPFA fills [0, 2) (beyond the Q1 bound 1.5), and the cycle
    on [0.2, 2] is symmetric positive definite at contrast 1e6."""
    n = 8
    rng = np.random.default_rng(3)
    rho = np.where(rng.uniform(size=n ** 3) < 0.4, 1.0, 1e-3)
    g, h = _setup(n, 2, 2, rho=rho, kmin=1e-6)
    lam = sla.eigvalsh(h.A_csr.toarray(), np.diag(h.diag))
    assert lam.max() < 2.0 and lam.max() > 1.6
    Minv = np.column_stack([h.precondition(np.eye(g.nelem)[:, j]) for j in range(g.nelem)])
    assert np.abs(Minv - Minv.T).max() <= 1e-9 * np.abs(Minv).max()
    assert np.linalg.eigvalsh(0.5 * (Minv + Minv.T)).min() > 0


def tpfa_source(rho, f0=1.0, p=3):
    """eq. (material) heat source f0 (1 - x^p) per cell."""
    return f0 * (1.0 - np.asarray(rho) ** p)


@pytest.mark.parametrize("f0", [0.0, 1.0])
def test_sensitivity_matches_finite_differences(f0):
    """dc/drho of c = w^T t with A(rho) t = b(rho) (heat source f0 (1 - rho^3),
    T_D on the patch faces) against central differences of direct solves."""
    shape = (5, 6, 7)
    g = q1.Grid(7, 6, 5, lx=1.0, ly=0.8, lz=1.2)
    rho = synth.uniform_noise_rho(7, 3, base=0.5, amp=0.3, shape=shape).ravel()
    flags = synth.dirichlet_patch_faces(7, 6, 5, frac=(1, 2)).ravel().astype(np.uint8)
    flags[g.element_index(6, 2, 3)] |= np.uint8(2)   # and one +x face
    kmin, kmax, p, td = 1e-2, 1.0, 3, 100.0
    wgt = np.random.default_rng(1).uniform(0.5, 1.5, g.nelem)
    src = np.random.default_rng(2).uniform(0.5, 1.5, g.nelem)

    def objective(r):
        k = q1.conductivity(r, kmin, kmax, p)
        f = tpfa.cell_load(g, src + f0 * (1.0 - r ** 3))
        t = tpfa.solve_direct(g, k, flags, f, td)
        return wgt @ t, t, k

    c0, t, k = objective(rho)
    lam = tpfa.solve_direct(g, k, flags, wgt, None)
    grad = tpfa.sensitivity(g, rho, t, lam, kmin, kmax, p, flags, td, f0)
    eps = 1e-4   # central differences: O(eps^2) truncation, far above the rounding of c ~ 1e4
    for K in (0, g.element_index(3, 3, 0), g.element_index(6, 2, 3), g.element_index(2, 4, 4), g.nelem - 1):
        rp, rm = rho.copy(), rho.copy()
        rp[K] += eps
        rm[K] -= eps
        fd = (objective(rp)[0] - objective(rm)[0]) / (2 * eps)
        assert abs(fd - grad[K]) <= 1e-6 * max(abs(fd), 1e-3 * abs(c0)), (K, fd, grad[K])


def test_adaptive_local_counts_match_brute_force():
    """The adaptive count l_c^i on TPFA cells: eigenvalues at or below
    thr * (pi / (H h))^2 of the full local spectrum, at least one, at most Lc."""
    n = 16
    rho = synth.grf_rho(n, 3, seed=4).ravel()
    g = q1.Grid(n)
    flags = synth.dirichlet_patch_faces(n, n, n).ravel()
    thr = 1.5
    h = tpfa.Hierarchy(g, rho, 1e-6, 1.0, 3, flags, tpfa.default_options(H=4, sd=2, Lc=6, lc_threshold=thr))
    theta = thr * (np.pi / (4 * g.hx)) ** 2
    counts = []
    for ci, (cx, cy, cz) in enumerate(h.cells):
        K, m, _ = h.local_problem(cx, cy, cz)
        lam = sla.eigh(K, np.diag(m), eigvals_only=True)
        want = min(6, max(1, int(np.count_nonzero(lam <= theta))))
        assert len(h.cell_rows[ci]) == want
        counts.append(want)
    assert min(counts) < max(counts) and h.n_c == sum(counts)
    f = tpfa.cell_load(g, 1.0 - rho ** 3)
    t, res, _ = tpfa.solve(g, rho, f, flags, 1e-6, 1.0, 3, hier=h, rtol=1e-10, td=100.0)
    td = tpfa.solve_direct(g, h.k, flags, f, 100.0)
    assert res.status == "converged" and np.linalg.norm(t - td) / np.linalg.norm(td) <= 1e-6
