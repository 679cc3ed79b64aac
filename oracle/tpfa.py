"""Oracle, part 5: the cell-centred two-point flux (TPFA) finite volumes of the
paper's own discretisation, and the three-grid preconditioner on them.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain FP64 code that
writes out the definitions; the operator is assembled face by face into a
sparse matrix.

What the paper fixes (section 2.2):
  * one unknown t_K per cell K of the structured mesh, the same indexing as
    the design variables;
  * eq. (flux): on an internal face F between cells K and L along axis d the
    flux is v_F = -kappa_F (t_L - t_K) / h_d with the harmonic mean
    kappa_F = 2 / (1/kappa_K + 1/kappa_L);
  * eq. (new linear system): assembling the cell balances sum_F |F| v_F . n =
    f_K |K| gives A t = f.
Section 3, eq. (spepb) and eq. (spectral cc), sum kappa_F times the products of
the face jumps over the faces internal to a coarse (coarse-coarse) cell, times
h_x h_y h_z, on the left, and integrate kappa Phi q over the cell on the right.

Readings taken where the paper is silent (each is also listed in the design
notes):
  * a Dirichlet face of Gamma_D (only boundary faces can carry one) closes the
    cell balance with the half-cell distance: v_F = -kappa_K (T_D - t_K) /
    (h_d / 2), so it adds 2 kappa_K |F| / h_d to the diagonal and that times
    T_D to the right-hand side; faces of Gamma_N carry no flux;
  * the load of cell K is f_K |K| (the cell integral of a cell-wise constant
    source);
  * local and coarse-coarse problems use the internal faces only, so Dirichlet
    faces never enter them (they are boundary faces), and no unknown is
    removed: every cell stays free;
  * coarse cells: along each axis the cells 0..N-1 are cut into runs of H, the
    last run keeps the remainder (the cells partition exactly, unlike the
    nodal reading of the Q1 solver); coarse-coarse cells group sd^3 coarse
    cells as there;
  * the coarse-coarse stiffness keeps the faces whose two cells lie in one
    coarse-coarse cell;
  * the level-0 smoother is Chebyshev-Jacobi as for Q1, on the interval
    [0.2, 2] that holds the spectrum of D^-1 A for TPFA (default_options).

Face flags (one byte per cell, the Dirichlet faces of that cell):
bit 0 the -x face, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z.
Cells are numbered (k ny + j) nx + i, x fastest (the element numbering of q1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import msmg, q1

FACE_BITS = ((0, -1, 0), (0, 1, 1), (1, -1, 2), (1, 1, 3), (2, -1, 4), (2, 1, 5))  # (axis, side, bit)


def cell_coords(grid):
    return grid.element_coords()


def _spacing(grid):
    return (grid.hx, grid.hy, grid.hz)


def face_weight(grid, axis):
    """|F| / h_d for a face normal to axis d: the transmissibility per unit kappa."""
    h = _spacing(grid)
    area = h[(axis + 1) % 3] * h[(axis + 2) % 3]
    return area / h[axis]


def harmonic_mean(ka, kb):
    """eq. (flux): kappa_F = 2 / (1/kappa_K + 1/kappa_L)."""
    return 2.0 / (1.0 / ka + 1.0 / kb)


def internal_faces(grid, axis, keep=None):
    """Cell pairs (K, L) across the internal faces normal to `axis` (L = K + e_axis).

    ``keep(i, j, k, axis)`` optionally filters faces by the lower cell's
    coordinates (used for the coarse-coarse restriction)."""
    ex, ey, ez = cell_coords(grid)
    n = (grid.nx, grid.ny, grid.nz)
    c = (ex, ey, ez)
    sel = c[axis] < n[axis] - 1
    if keep is not None:
        sel &= keep(ex, ey, ez, axis)
    K = np.flatnonzero(sel)
    step = (1, grid.nx, grid.nx * grid.ny)[axis]
    return K, K + step


def check_face_flags(grid, dface):
    """Raise unless every flagged face lies on the domain boundary."""
    dface = np.asarray(dface).ravel().astype(np.int64)
    if dface.shape[0] != grid.nelem:
        raise ValueError("one flag byte per cell")
    ex, ey, ez = cell_coords(grid)
    c = (ex, ey, ez)
    n = (grid.nx, grid.ny, grid.nz)
    if (dface & ~63).any():
        raise ValueError("face flags use bits 0..5 only")
    for axis, side, bit in FACE_BITS:
        on = (dface >> bit) & 1
        boundary = (c[axis] == 0) if side < 0 else (c[axis] == n[axis] - 1)
        if (on.astype(bool) & ~boundary).any():
            raise ValueError("a Dirichlet flag sits on an internal face")
    return dface


def dirichlet_weight(grid, kcell, dface):
    """Per cell: sum over its Dirichlet faces of 2 kappa_K |F| / h_d (the reading above)."""
    dface = check_face_flags(grid, dface)
    w = np.zeros(grid.nelem)
    for axis, side, bit in FACE_BITS:
        on = ((dface >> bit) & 1).astype(np.float64)
        w += on * 2.0 * kcell * face_weight(grid, axis)
    return w


def assemble(grid, kcell, dface=None, keep=None, dirichlet=True):
    """A of eq. (new linear system): sum over internal faces of T_F (e_K - e_L)(e_K - e_L)^T
    plus the Dirichlet faces' diagonal; scipy CSR over the cells.

    ``keep`` restricts the internal faces (see internal_faces); dirichlet=False
    drops the Dirichlet diagonal (the local problems' Neumann forms)."""
    kcell = np.asarray(kcell, dtype=np.float64).ravel()
    rows, cols, vals = [], [], []
    for axis in range(3):
        K, L = internal_faces(grid, axis, keep)
        T = face_weight(grid, axis) * harmonic_mean(kcell[K], kcell[L])
        rows += [K, L, K, L]
        cols += [K, L, L, K]
        vals += [T, T, -T, -T]
    n = grid.nelem
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    if dirichlet and dface is not None:
        A = (A + sp.diags(dirichlet_weight(grid, kcell, dface))).tocsr()
    return A


def cell_load(grid, source):
    """Load of eq. (new linear system): f_K |K| for a cell-wise constant source (array or scalar)."""
    s = np.broadcast_to(np.asarray(source, dtype=np.float64), (grid.nelem,)) if np.ndim(source) == 0 \
        else np.asarray(source, dtype=np.float64).ravel()
    return s * grid.vol


def rhs(grid, kcell, dface, f, td=None):
    """b = f + sum over Dirichlet faces of 2 kappa_K |F| / h_d T_D (td per cell, or None = 0)."""
    b = np.asarray(f, dtype=np.float64).ravel().copy()
    if td is None:
        return b
    tdv = np.broadcast_to(np.asarray(td, dtype=np.float64), (grid.nelem,)) if np.ndim(td) == 0 \
        else np.asarray(td, dtype=np.float64).ravel()
    return b + dirichlet_weight(grid, kcell, dface) * tdv


def solve_direct(grid, kcell, dface, f, td=None):
    """t = A^-1 b by sparse LU (needs at least one Dirichlet face)."""
    if not np.asarray(dface).any():
        raise ValueError("no Dirichlet face: the operator is singular")
    A = assemble(grid, kcell, dface)
    return spla.spsolve(A.tocsc(), rhs(grid, kcell, dface, f, td))


class Operator:
    """y = A x in difference form: sum_F T_F (x_K - x_L) plus the Dirichlet diagonal.

    The same matrix as ``assemble``; the internal faces enter through
    neighbour differences, so the rounding follows the local variation of x
    rather than its size (T reaches ~1/k_min on low-conductivity islands).
    """

    def __init__(self, grid, kcell, dface):
        kcell = np.asarray(kcell, dtype=np.float64).ravel()
        r, c, v = [], [], []
        for axis in range(3):
            K, L = internal_faces(grid, axis)
            T = face_weight(grid, axis) * harmonic_mean(kcell[K], kcell[L])
            r += [K, L]
            c += [L, K]
            v += [T, T]
        self.r = np.concatenate(r)
        self.c = np.concatenate(c)
        self.v = np.concatenate(v)
        self.wd = dirichlet_weight(grid, kcell, dface) if dface is not None else np.zeros(grid.nelem)
        self.n = grid.nelem
        self.shape = (self.n, self.n)

    def __matmul__(self, x):
        x = np.asarray(x, dtype=np.float64)
        y = np.bincount(self.r, weights=self.v * (x[self.r] - x[self.c]), minlength=self.n)
        return y + self.wd * x

    def free_product(self, x):
        """A x for x of any float precision: neighbour differences and the
        Dirichlet term are formed in the precision of x, then rounded."""
        d = (x[self.r] - x[self.c]).astype(np.float64)
        y = np.bincount(self.r, weights=self.v * d, minlength=self.n)
        return y + (self.wd.astype(x.dtype) * x).astype(np.float64)


def default_options(**kw):
    """Options of the three-grid cycle for TPFA: Chebyshev-Jacobi on [0.2, 2].

    The Jacobi-scaled TPFA matrix D^-1 A has its spectrum in [0, 2] (its
    off-diagonal row sums never exceed the diagonal) and reaches close to 2
    on oscillating modes, so the smoothing interval must end at 2 (the Q1
    interval ending at 1.5 amplifies those modes and makes the cycle
    indefinite); the lower end keeps the Q1 ratio hi / lo = 10."""
    o = dict(cheb_lo=0.2, cheb_hi=2.0)
    o.update(kw)
    return msmg.Options(**o)


def sensitivity(grid, rho, t, lam, kmin, kmax, p, dface, td=None, f0=0.0):
    """dc/drho_K = lam^T (db/drho_K - dA/drho_K t) for A(rho) t = b(rho) and an
    objective c with adjoint A lam = dc/dt (section 2.3), on TPFA:

      * internal face F = (K, L): T_F = w_d 2 k_K k_L / (k_K + k_L), so
        dT_F/dk_K = w_d 2 k_L^2 / (k_K + k_L)^2 and the face adds
        -dT_F/dk_K (lam_K - lam_L)(t_K - t_L);
      * Dirichlet face of K: 2 w_d k_K on the diagonal and in the right-hand
        side (times T_D), adding 2 w_d lam_K (T_D - t_K);
      * both times dk/drho = p rho^(p-1) (k_max - k_min);
      * the heat source f0 (1 - rho^p) |K| adds lam_K (-f0 p rho^(p-1)) |K|.
    td: per-cell Dirichlet values (None = 0)."""
    rho = np.asarray(rho, dtype=np.float64).ravel()
    t = np.asarray(t, dtype=np.float64).ravel()
    lam = np.asarray(lam, dtype=np.float64).ravel()
    k = q1.conductivity(rho, kmin, kmax, p)
    g = np.zeros(grid.nelem)
    for axis in range(3):
        K, L = internal_faces(grid, axis)
        w = face_weight(grid, axis)
        s2 = (k[K] + k[L]) ** 2
        prod = (lam[K] - lam[L]) * (t[K] - t[L])
        np.add.at(g, K, -w * 2.0 * k[L] ** 2 / s2 * prod)
        np.add.at(g, L, -w * 2.0 * k[K] ** 2 / s2 * prod)
    dface = check_face_flags(grid, dface)
    tdv = np.zeros(grid.nelem) if td is None else np.broadcast_to(np.asarray(td, dtype=np.float64),
                                                                 (grid.nelem,)).copy()
    for axis, side, bit in FACE_BITS:
        on = ((dface >> bit) & 1).astype(np.float64)
        g += on * 2.0 * face_weight(grid, axis) * lam * (tdv - t)
    rp1 = np.ones_like(rho)
    for _ in range(int(p) - 1):
        rp1 = rp1 * rho
    g *= p * rp1 * (kmax - kmin)
    if f0:
        g += lam * (-f0 * p * rp1) * grid.vol
    return g


def cell_runs(n_cells, H):
    """Cell runs along one axis: [(start, end_exclusive)] over cells 0..n_cells-1."""
    nc = n_cells // H
    if nc < 1 or H < 2:
        raise ValueError("need H >= 2 and at least H cells per axis")
    starts = [c * H for c in range(nc)]
    ends = starts[1:] + [n_cells]
    return list(zip(starts, ends))


class Hierarchy(msmg.Hierarchy):
    """The three-grid hierarchy of section 3 on TPFA unknowns.

    Level 1 solves eq. (spepb) on every coarse cell: the TPFA form of the
    faces internal to the cell against the diagonal kappa_K |K|; level 2 solves
    eq. (spectral cc) in W_c with the faces internal to each coarse-coarse cell.
    Everything else (Galerkin operators, smoothers, Algorithm 1) is the Q1
    solver's, acting on these matrices.
    """

    def __init__(self, grid, rho, kmin, kmax, p, dface, opts=None, keep_local=True):
        self.g = grid
        self.o = opts or default_options()
        self.kmin, self.kmax, self.p = kmin, kmax, p
        self.n_unknowns = grid.nelem
        self.dface = check_face_flags(grid, dface)
        self.mask = np.zeros(grid.nelem, dtype=bool)   # no unknown is fixed
        self.k = q1.conductivity(np.asarray(rho).ravel(), kmin, kmax, p)
        self.A_csr = assemble(grid, self.k, self.dface)
        self.A = Operator(grid, self.k, self.dface)
        self.diag = self.A_csr.diagonal().copy()
        self._partition()
        self._level1(keep_local)
        self._level2()

    def _axis_runs(self, axis):
        return cell_runs((self.g.nx, self.g.ny, self.g.nz)[axis], self.o.H)

    def _axis_unknowns(self):
        return (self.g.nx, self.g.ny, self.g.nz)

    def unknown_index(self, i, j, k):
        return self.g.element_index(i, j, k)

    def local_problem(self, cx, cy, cz):
        """eq. (spepb) on one coarse cell: TPFA form of its internal faces, mass kappa_K |K|."""
        g = self.g
        (sx, ex), (sy, ey), (sz, ez) = self.runs[0][cx], self.runs[1][cy], self.runs[2][cz]
        nodes = self.cell_nodes(cx, cy, cz)
        lx, ly, lz = ex - sx, ey - sy, ez - sz
        nl = len(nodes)
        kl = self.k[nodes]
        K = np.zeros((nl, nl))
        for axis, (step, nax) in enumerate(((1, lx), (lx, ly), (lx * ly, lz))):
            li = np.arange(nl)
            pos = (li % lx, (li // lx) % ly, li // (lx * ly))[axis]
            a = li[pos < nax - 1]
            b = a + step
            T = face_weight(g, axis) * harmonic_mean(kl[a], kl[b])
            np.add.at(K, (a, a), T)
            np.add.at(K, (b, b), T)
            np.add.at(K, (a, b), -T)
            np.add.at(K, (b, a), -T)
        m = kl * g.vol
        return K, m, nodes

    def cc_stiffness(self):
        """TPFA form of the faces whose two cells share a coarse-coarse cell (no Dirichlet part)."""
        own, grp = self.own_axis, self.grp_axis

        def keep(ex, ey, ez, axis):
            c = (ex, ey, ez)
            lo = grp[axis][own[axis][c[axis]]]
            nmax = own[axis].shape[0] - 1
            hi = grp[axis][own[axis][np.minimum(c[axis] + 1, nmax)]]
            return lo == hi

        return assemble(self.g, self.k, None, keep=keep, dirichlet=False)


def solve(grid, rho, f, dface, kmin, kmax, p, opts=None, rtol=1e-8, maxit=1000, td=None, hier=None):
    """t from PCG with the three-grid preconditioner; returns (t, PCGResult, Hierarchy)."""
    h = hier or Hierarchy(grid, rho, kmin, kmax, p, dface, opts)
    b = rhs(grid, h.k, h.dface, f, td)
    res = msmg.pcg(h.A, b, h.precondition, rtol=rtol, maxit=maxit)
    return res.x.copy(), res, h
