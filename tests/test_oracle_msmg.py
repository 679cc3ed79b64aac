"""Pins of the oracle's multiscale multigrid preconditioner and PCG (CPU only).

Pins: closed-form local eigenpairs at constant conductivity, the
normalisation invariant R_c M R_c^T = I, exactness with full coarse spaces,
the explicit error-propagation formula of the three-grid cycle, the
closed-form Chebyshev error polynomial, symmetry / positivity / basis
invariance of the preconditioner, and agreement of PCG with direct solves.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import msmg, q1


def _cheb_T(d, x):
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(d * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** d * np.cosh(d * np.arccosh(np.abs(xo)))
    return out


def _closed_form_evals(nx, ny, nz, hx, hy, hz):
    """All eigenvalues of the constant-k local Neumann problem with lumped mass."""
    def lam_s(j, n, h):
        return (2.0 / h) * (1.0 - np.cos(j * np.pi / n))

    def lam_m(j, n, h):
        return (h / 3.0) * (2.0 + np.cos(j * np.pi / n))

    a = np.arange(nx + 1)[:, None, None]
    b = np.arange(ny + 1)[None, :, None]
    c = np.arange(nz + 1)[None, None, :]
    lam = (lam_s(a, nx, hx) * lam_m(b, ny, hy) * lam_m(c, nz, hz)
           + lam_m(a, nx, hx) * lam_s(b, ny, hy) * lam_m(c, nz, hz)
           + lam_m(a, nx, hx) * lam_m(b, ny, hy) * lam_s(c, nz, hz)) / (hx * hy * hz)
    return np.sort(lam.ravel())


def _setup(n, H, sd, Lc=4, Lcc=17, rho=None, kmin=1e-3, seed=0, mask=None, deg=2):
    g = q1.Grid(n)
    rho = synth.uniform_noise_rho(n, seed).ravel() if rho is None else rho
    mask = synth.dirichlet_patch_mask(n, n, n).ravel() if mask is None else mask
    h = msmg.Hierarchy(g, rho, kmin, 1.0, 3, mask,
                       msmg.Options(H=H, sd=sd, Lc=Lc, Lcc=Lcc, cheb_degree=deg))
    return g, h


def test_partition_is_exact():
    for n, H in [(16, 8), (17, 8), (12, 4), (9, 2), (8, 8)]:
        runs = msmg.axis_runs(n, H)
        covered = np.concatenate([np.arange(s, e) for s, e in runs])
        assert np.array_equal(covered, np.arange(n + 1))
        assert all(e - s >= H for s, e in runs)
    for nc, sd in [(32, 8), (5, 2), (1, 8), (7, 3)]:
        gr = msmg.axis_groups(nc, sd)
        covered = np.concatenate([np.arange(s, e) for s, e in gr])
        assert np.array_equal(covered, np.arange(nc))


def test_shell_multiplicities_of_default_sizes():
    """L_c = 4 and L_cc = 17 sit at complete degenerate shells (boxes of 7 and 8 elements)."""
    for n in (7, 8):
        lam = _closed_form_evals(n, n, n, 1.0, 1.0, 1.0)
        gaps = np.flatnonzero(np.diff(lam[:20]) > 1e-9 * lam[20])
        cum = list(gaps + 1)
        for want in (1, 4, 7, 8, 11, 17):
            assert want in cum, (n, cum)


@pytest.mark.parametrize("rhoval", [1.0, 0.5])
def test_local_eigenpairs_constant_k_closed_form(rhoval):
    n = 16
    g, h = _setup(n, 8, 2, Lc=8, rho=np.full(n ** 3, rhoval))
    checked = 0
    for ci, (cx, cy, cz) in enumerate(h.cells):
        nodes, phi = h.cell_basis[ci]
        (sx, ex), (sy, ey), (sz, ez) = h.runs[0][cx], h.runs[1][cy], h.runs[2][cz]
        if h.mask[h.cell_nodes(cx, cy, cz)].any():
            assert h.cell_evals[ci][0] > 1e-6   # fixed nodes remove the constant mode
            continue
        want = _closed_form_evals(ex - sx - 1, ey - sy - 1, ez - sz - 1, g.hx, g.hy, g.hz)[:8]
        got = h.cell_evals[ci]
        assert abs(got[0]) <= 1e-10 * want[-1]
        assert np.allclose(got[1:], want[1:], rtol=1e-12, atol=0)
        checked += 1
    assert checked >= 4


def test_local_basis_normalisation_and_supports():
    n = 16
    g, h = _setup(n, 4, 2, kmin=1e-6, rho=synth.grf_rho(n, 4, seed=1).ravel())
    owner = np.full(g.nnodes, -1)
    for ci in range(len(h.cells)):
        nodes, phi = h.cell_basis[ci]
        m = h.cell_mass[ci]
        G = phi.T @ (m[:, None] * phi)
        assert np.allclose(G, np.eye(phi.shape[1]), atol=1e-12)
        assert (owner[nodes] == -1).all()
        owner[nodes] = ci
        assert not h.mask[nodes].any()
    # R_c rows carry exactly these vectors
    Rc = h.Rc.toarray()
    for ci in range(len(h.cells)):
        nodes, phi = h.cell_basis[ci]
        assert np.array_equal(Rc[np.ix_(h.cell_rows[ci], nodes)], phi.T)


def test_cc_level_invariants():
    n = 16
    g, h = _setup(n, 4, 2, rho=np.full(n ** 3, 1.0), mask=np.zeros(17 ** 3, dtype=np.uint8))
    # no fixed nodes: the constant lies in W_c and in the kernel of every cc stiffness
    for lam in h.cc_evals:
        assert abs(lam[0]) <= 1e-9 * max(1.0, abs(lam[-1]))
    Rcc = h.Rcc.toarray()
    assert np.allclose(Rcc @ Rcc.T, np.eye(h.n_cc), atol=1e-12)


def test_galerkin_identity():
    g, h = _setup(8, 2, 2, Lc=3, Lcc=5)
    P = (h.Rcc @ h.Rc).toarray()
    A = h.A_csr.toarray()
    assert np.allclose(h.Acc, P @ A @ P.T, rtol=0, atol=1e-12 * np.abs(h.Acc).max())
    assert np.all(np.linalg.eigvalsh(h.Acc) > 0)


def test_full_coarse_spaces_make_one_iteration():
    n = 4
    g, h = _setup(n, 2, 1, Lc=27, Lcc=10 ** 6)
    f = q1.element_load(g, 1.0)
    T, res, _ = msmg.solve(g, None, f, h.mask, 1e-3, 1.0, 3, hier=h, rtol=1e-10)
    assert res.iterations == 1 and res.status == "converged"


def _free(h):
    return np.flatnonzero(~h.mask)


def _chebyshev_matrix(A, D, o):
    """S^-1 = V diag(q(lam)) V^T with 1 - lam q(lam) = T_d((theta-lam)/delta) / T_d(theta/delta)."""
    lam, V = sla.eigh(A, np.diag(D))       # A V = D V Lam, V^T D V = I
    theta = 0.5 * (o.cheb_hi + o.cheb_lo)
    delta = 0.5 * (o.cheb_hi - o.cheb_lo)
    err = _cheb_T(o.cheb_degree, (theta - lam) / delta) / _cheb_T(o.cheb_degree, np.array([theta / delta]))[0]
    q = (1.0 - err) / lam
    return V @ np.diag(q) @ V.T


@pytest.mark.parametrize("deg", [1, 2, 3, 5])
def test_chebyshev_error_polynomial(deg):
    g, h = _setup(6, 2, 2, deg=deg)
    F = _free(h)
    A = h.A_csr.toarray()[np.ix_(F, F)]
    D = h.diag[F]
    lam, V = sla.eigh(A, np.diag(D))
    o = h.o
    theta, delta = 0.5 * (o.cheb_hi + o.cheb_lo), 0.5 * (o.cheb_hi - o.cheb_lo)
    for j in (0, len(lam) // 3, len(lam) - 1):
        v = np.zeros(g.nnodes)
        v[F] = V[:, j]
        Av = h.A @ v
        got = v - h.chebyshev(Av)
        want = _cheb_T(deg, np.array([(theta - lam[j]) / delta]))[0] / \
            _cheb_T(deg, np.array([theta / delta]))[0]
        assert np.abs(got[F] - want * V[:, j]).max() <= 1e-11 * np.abs(V[:, j]).max()


def test_smoother_interval_upper_bound():
    rng = np.random.default_rng(2)
    n = 6
    rho = np.where(rng.uniform(size=n ** 3) < 0.4, 1.0, 1e-3)
    g, h = _setup(n, 2, 2, rho=rho, kmin=1e-6)
    F = _free(h)
    lam = sla.eigvalsh(h.A_csr.toarray()[np.ix_(F, F)], np.diag(h.diag[F]))
    assert lam.max() <= 1.5 * (1 + 1e-12)
    assert lam.max() > 1.2


def test_three_grid_error_propagation_formula():
    """I - M^-1 A = (I - S^-T A)(I - R_c^T B_c R_c A)(I - S^-1 A), with
    I - B_c A_c = (I - S_c^-T A_c)(I - R_cc^T A_cc^-1 R_cc A_c)(I - S_c^-1 A_c),
    S = Chebyshev polynomial (closed form), S_c = block lower triangle of A_c in colour order."""
    g, h = _setup(6, 2, 2, Lc=4, Lcc=17)
    F = _free(h)
    nf = len(F)
    A = h.A_csr.toarray()[np.ix_(F, F)]
    Sinv = _chebyshev_matrix(A, h.diag[F], h.o)
    Rc = h.Rc.toarray()[:, F]
    Ac = h.Ac.toarray()
    blk = np.empty(h.n_c, dtype=np.int64)
    for ci, rows in enumerate(h.cell_rows):
        blk[rows] = ci
    col = np.array([h.colour(*h.cells[b]) for b in blk])
    # S_c = D + L: keep (i, j) when j sits in i's block or in an earlier colour of the sweep
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
    Minv = np.zeros((nf, nf))
    for j in range(nf):
        e = np.zeros(g.nnodes)
        e[F[j]] = 1.0
        Minv[:, j] = h.precondition(e)[F]
    assert np.abs(Minv - Minv_formula).max() <= 1e-10 * np.abs(Minv).max()


def test_preconditioner_symmetric_positive():
    g, h = _setup(16, 4, 2, kmin=1e-6, rho=synth.grf_rho(16, 4, seed=2).ravel())
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, g.nnodes))
    x[h.mask] = 0
    y[h.mask] = 0
    mx, my = h.precondition(x), h.precondition(y)
    assert abs(mx @ y - x @ my) <= 1e-11 * abs(mx @ y)
    assert mx @ x > 0 and my @ y > 0


def test_preconditioner_basis_invariance():
    g, h = _setup(16, 4, 2, kmin=1e-4, rho=synth.grf_rho(16, 4, seed=3).ravel())
    r = np.random.default_rng(1).standard_normal(g.nnodes)
    r[h.mask] = 0
    y0 = h.precondition(r)
    rng = np.random.default_rng(7)
    Q = np.zeros((h.n_c, h.n_c))
    for rows in h.cell_rows:
        q, _ = np.linalg.qr(rng.standard_normal((len(rows), len(rows))))
        Q[np.ix_(rows, rows)] = q
    import scipy.sparse as sp
    h.Rc = sp.csr_matrix(Q @ h.Rc.toarray())
    h.level1_operators()
    h.Rcc = sp.csr_matrix(h.Rcc.toarray() @ Q.T)
    h.level2_operators()
    y1 = h.precondition(r)
    assert np.abs(y1 - y0).max() <= 1e-11 * np.abs(y0).max()


@pytest.mark.parametrize("n,H,sd", [(8, 2, 2), (8, 4, 1), (16, 8, 2), (16, 4, 2), (12, 4, 8)])
def test_pcg_msmg_matches_direct_solve(n, H, sd):
    g = q1.Grid(n)
    rho = synth.uniform_noise_rho(n, 0).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    f = q1.element_load(g, 1.0)
    T, res, h = msmg.solve(g, rho, f, mask, 1e-3, 1.0, 3, msmg.Options(H=H, sd=sd), rtol=1e-12)
    assert res.status == "converged" and res.rel_res <= 1e-12
    Td = q1.solve_direct(q1.assemble(g, h.k), f, mask)
    assert np.linalg.norm(T - Td) / np.linalg.norm(Td) <= 1e-10
    assert res.iterations <= 30


def test_pcg_high_contrast_and_warm_start():
    n = 16
    g = q1.Grid(n)
    rho = synth.grf_rho(n, 4, seed=0).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    f = q1.element_load(g, 1.0)
    T, res, h = msmg.solve(g, rho, f, mask, 1e-6, 1.0, 3, msmg.Options(H=4, sd=2), rtol=1e-8)
    A = q1.assemble(g, h.k)
    assert res.status == "converged"
    assert q1.relative_residual(A, T, f, mask) <= 1e-8
    # warm start from the solution converges immediately
    T2, res2, _ = msmg.solve(g, rho, f, mask, 1e-6, 1.0, 3, hier=h, rtol=1e-8, x0=T)
    assert res2.iterations == 0
    # deterministic
    T3, res3, _ = msmg.solve(g, rho, f, mask, 1e-6, 1.0, 3, hier=h, rtol=1e-8)
    assert res3.iterations == res.iterations and np.array_equal(T3, T)


def test_extended_iterate_beats_binary64_floor():
    """At contrast 1e6 a binary64 T cannot reach 1e-8; the extended iterate can."""
    n = 16
    g = q1.Grid(n)
    rho = synth.grf_rho(n, 4, seed=2).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    f = q1.element_load(g, 1.0)
    A = q1.assemble(g, q1.conductivity(rho, 1e-6, 1.0, 3))
    Td = q1.solve_direct(A, f, mask)
    assert q1.relative_residual_diff(A, Td, f, mask) > 1e-9      # binary64 floor of this field
    T, res, h = msmg.solve(g, rho, f, mask, 1e-6, 1.0, 3, msmg.Options(H=4, sd=2), rtol=1e-10, maxit=300)
    assert res.status == "converged"
    assert q1.relative_residual_diff(A, T, f, mask, T_lo=res.x_lo) <= 1e-10 * (1 + 1e-3)


@pytest.mark.parametrize("thr", [1.0, 2.5])
def test_adaptive_local_counts_match_brute_force(thr):
    """With lc_threshold each cell keeps its eigenpairs at or below
    thr * (pi / (H h))^2 (at least one, at most Lc): checked against the full
    dense spectrum of every local problem; the cycle stays SPD and PCG
    reaches the direct solution."""
    n = 16
    rho = synth.grf_rho(n, 3, seed=4).ravel()
    g, h = _setup(n, 4, 2, Lc=6, rho=rho, kmin=1e-6)
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    ha = msmg.Hierarchy(g, rho, 1e-6, 1.0, 3, mask, msmg.Options(H=4, sd=2, Lc=6, lc_threshold=thr))
    theta = thr * (np.pi / (4 * g.hx)) ** 2
    counts = []
    for ci, (cx, cy, cz) in enumerate(ha.cells):
        K, m, _ = ha.local_problem(cx, cy, cz)
        lam = sla.eigh(K, np.diag(m), eigvals_only=True)
        want = min(6, max(1, int(np.count_nonzero(lam <= theta))))
        assert len(ha.cell_rows[ci]) == want, (ci, lam[:8], theta)
        assert np.allclose(ha.cell_evals[ci], h.cell_evals[ci][:want], rtol=1e-10, atol=1e-10 * lam[-1])
        counts.append(want)
    assert min(counts) < max(counts)  # the field makes the counts differ between cells
    assert ha.n_c == sum(counts) < h.n_c
    x, y = np.random.default_rng(0).standard_normal((2, g.nnodes))
    x[ha.mask] = 0
    y[ha.mask] = 0
    mx, my = ha.precondition(x), ha.precondition(y)
    assert abs(mx @ y - x @ my) <= 1e-11 * abs(mx @ y)
    assert mx @ x > 0
    f = q1.element_load(g, 1.0)
    T, res, _ = msmg.solve(g, rho, f, mask, 1e-6, 1.0, 3, hier=ha, rtol=1e-10)
    Td = q1.solve_direct(q1.assemble(g, ha.k), f, mask)
    assert res.status == "converged" and np.linalg.norm(T - Td) / np.linalg.norm(Td) <= 1e-6
