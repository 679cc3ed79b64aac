"""Oracle, part 1: the Q1 discretisation of the state and adjoint problems.

TEST INFRASTRUCTURE ONLY (see the package docstring): plain, slow FP64 code
that writes out the definitions.  The operator is assembled by scattering
element matrices into a sparse matrix; it never uses a node stencil.

Paper anchors
  * material law, section 2.1 eq. (material): k = k_L + x^p (k_H - k_L);
  * the linear system A t = f, section 2.2 eq. (new linear system), here with
    trilinear (Q1) hexahedral elements instead of the paper's two-point flux
    finite volumes (the nodal reading is the one this project solves);
  * adjoint sensitivity, section 2.3, eq. (adjoint): A u = dc/dt and
    dc/dx = u^T (df/dx - dA/dx t), with df/dx = 0 for a fixed source and
    df/dx from eq. (material) for the design-dependent heat source f0 (1 - x^p);
  * mean-temperature objective, section 2.3 eq. (cost function).

Layouts: nodes n = (k (ny+1) + j)(nx+1) + i, elements e = (k ny + j) nx + i
(x fastest); element-local node a = ax + 2 ay + 4 az.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class Grid:
    """Structured box mesh of nx * ny * nz trilinear hexahedra."""

    def __init__(self, nx, ny=None, nz=None, lx=1.0, ly=1.0, lz=1.0):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.lx, self.ly, self.lz = float(lx), float(ly), float(lz)
        self.hx = self.lx / self.nx
        self.hy = self.ly / self.ny
        self.hz = self.lz / self.nz
        self.vol = self.hx * self.hy * self.hz
        self.nnx, self.nny, self.nnz = self.nx + 1, self.ny + 1, self.nz + 1
        self.nnodes = self.nnx * self.nny * self.nnz
        self.nelem = self.nx * self.ny * self.nz

    def node_index(self, i, j, k):
        return (k * self.nny + j) * self.nnx + i

    def element_index(self, i, j, k):
        return (k * self.ny + j) * self.nx + i

    def element_coords(self):
        ez, ey, ex = np.meshgrid(np.arange(self.nz), np.arange(self.ny),
                                 np.arange(self.nx), indexing="ij")
        return ex.ravel(), ey.ravel(), ez.ravel()

    def node_coords(self):
        kz, jy, ix = np.meshgrid(np.arange(self.nnz), np.arange(self.nny),
                                 np.arange(self.nnx), indexing="ij")
        return ix.ravel(), jy.ravel(), kz.ravel()

    def element_nodes(self, elems=None):
        """(nelem, 8) global node ids of each element, local order ax + 2 ay + 4 az."""
        ex, ey, ez = self.element_coords()
        if elems is not None:
            ex, ey, ez = ex[elems], ey[elems], ez[elems]
        cols = []
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            cols.append(self.node_index(ex + ax, ey + ay, ez + az))
        return np.stack(cols, axis=1)


_S1 = np.array([[1.0, -1.0], [-1.0, 1.0]])           # 1D stiffness on a unit interval
_M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0       # 1D consistent mass on a unit interval


def element_stiffness(hx, hy, hz):
    """Unit-conductivity Q1 stiffness K0 of an hx * hy * hz box (8 x 8).

    K0 = (hy hz / hx) S(x)M(x)M + (hx hz / hy) M(x)S(x)M + (hx hy / hz) M(x)M(x)S with the
    1D factors ordered z, y, x (the local node index is ax + 2 ay + 4 az).
    """
    kx = (hy * hz / hx) * np.kron(_M1, np.kron(_M1, _S1))
    ky = (hx * hz / hy) * np.kron(_M1, np.kron(_S1, _M1))
    kz = (hx * hy / hz) * np.kron(_S1, np.kron(_M1, _M1))
    return kx + ky + kz


def element_mass(hx, hy, hz):
    """Q1 consistent mass of an hx * hy * hz box (8 x 8)."""
    return np.kron(hz * _M1, np.kron(hy * _M1, hx * _M1))


def conductivity(rho, kmin, kmax, p):
    """Section 2.1 eq. (material): k = k_min + rho^p (k_max - k_min), rho^p by repeated products."""
    rho = np.asarray(rho, dtype=np.float64)
    rp = rho.copy()
    for _ in range(int(p) - 1):
        rp = rp * rho
    return kmin + rp * (kmax - kmin)


def assemble(grid, kelem, elems=None):
    """A = sum_e k_e K0_e (pure Neumann, all nodes), scipy CSR.

    ``elems`` optionally restricts the sum to a subset of elements.
    """
    kelem = np.asarray(kelem, dtype=np.float64).ravel()
    K0 = element_stiffness(grid.hx, grid.hy, grid.hz)
    en = grid.element_nodes(elems)
    ke = kelem if elems is None else kelem[elems]
    rows = np.repeat(en, 8, axis=1).ravel()
    cols = np.tile(en, (1, 8)).ravel()
    vals = (ke[:, None] * K0.ravel()[None, :]).ravel()
    n = grid.nnodes
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def assemble_mass(grid):
    """Consistent Q1 mass matrix (for manufactured-solution loads)."""
    M0 = element_mass(grid.hx, grid.hy, grid.hz)
    en = grid.element_nodes()
    rows = np.repeat(en, 8, axis=1).ravel()
    cols = np.tile(en, (1, 8)).ravel()
    vals = np.tile(M0.ravel(), grid.nelem)
    n = grid.nnodes
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def masked_operator(A, mask):
    """P A P + (I - P): the free-free block of A, identity on fixed nodes."""
    mask = np.asarray(mask).ravel().astype(bool)
    pf = sp.diags((~mask).astype(np.float64))
    return (pf @ A @ pf + sp.diags(mask.astype(np.float64))).tocsr()


def element_load(grid, source):
    """Consistent load of an element-wise constant source: f_n = sum_{e ni n} s_e V / 8."""
    s = np.broadcast_to(np.asarray(source, dtype=np.float64).ravel(), (grid.nelem,))
    en = grid.element_nodes()
    f = np.zeros(grid.nnodes)
    np.add.at(f, en.ravel(), np.repeat(s * grid.vol / 8.0, 8))
    return f


def element_load_rows(grid, source_const, nodes):
    """Rows of element_load for a constant source at the given nodes only:
    f_n = s V / 8 times the number of elements around n."""
    nodes = np.asarray(nodes, dtype=np.int64).ravel()
    i = nodes % grid.nnx
    j = (nodes // grid.nnx) % grid.nny
    k = nodes // (grid.nnx * grid.nny)
    cnt = np.zeros(nodes.size)
    for c in range(8):
        ex, ey, ez = i - 1 + (c & 1), j - 1 + ((c >> 1) & 1), k - 1 + ((c >> 2) & 1)
        cnt += ((ex >= 0) & (ex < grid.nx) & (ey >= 0) & (ey < grid.ny) & (ez >= 0) & (ez < grid.nz))
    return float(source_const) * grid.vol / 8.0 * cnt


def lifted_rhs(A, f, mask, td=None):
    """Right-hand side b of the masked system: b_F = f_F - A_FD T_D, b_D = T_D."""
    mask = np.asarray(mask).ravel().astype(bool)
    td = np.zeros(A.shape[0]) if td is None else np.asarray(td, dtype=np.float64).ravel()
    tfix = np.where(mask, td, 0.0)
    b = np.asarray(f, dtype=np.float64).ravel() - A @ tfix
    b[mask] = tfix[mask]
    return b


def solve_direct(A, f, mask, td=None):
    """T with T_D = td on fixed nodes and A_FF T_F = f_F - A_FD T_D (sparse LU)."""
    mask = np.asarray(mask).ravel().astype(bool)
    if not (~mask).any():
        raise ValueError("no free nodes")
    fr = np.flatnonzero(~mask)
    fx = np.flatnonzero(mask)
    if fx.size == 0:
        raise ValueError("empty Dirichlet set: the Neumann operator is singular")
    td = np.zeros(A.shape[0]) if td is None else np.asarray(td, dtype=np.float64).ravel()
    T = np.zeros(A.shape[0])
    T[fx] = td[fx]
    Aff = A[fr][:, fr].tocsc()
    rhs = np.asarray(f, dtype=np.float64).ravel()[fr] - A[fr][:, fx] @ td[fx]
    T[fr] = spla.spsolve(Aff, rhs)
    return T


def relative_residual(A, T, f, mask, td=None):
    """||(f - A T)_F||_2 / ||b_F||_2 with b the lifted right-hand side."""
    mask = np.asarray(mask).ravel().astype(bool)
    fr = ~mask
    res = (np.asarray(f).ravel() - A @ np.asarray(T).ravel())[fr]
    b = lifted_rhs(A, f, mask, td)[fr]
    return float(np.linalg.norm(res) / np.linalg.norm(b))


def compliance(f, T):
    """c = f^T T (equals the integral of T for f = 1 on the unit cube)."""
    return float(np.dot(np.asarray(f).ravel(), np.asarray(T).ravel()))


def adjoint_solve(A, g, mask):
    """Section 2.3 eq. (adjoint) restricted to free nodes: A_FF u_F = g_F, u_D = 0."""
    mask = np.asarray(mask).ravel().astype(bool)
    return solve_direct(A, np.asarray(g, dtype=np.float64).ravel(), mask,
                        np.zeros(A.shape[0]))


def sensitivity(grid, rho, T, lam, kmin, kmax, p):
    """dc/drho_e = -(dk/drho)_e lam_e^T K0 T_e  (section 2.3, df/drho = 0).

    dk/drho = p rho^(p-1) (k_max - k_min); lam is the adjoint (zero on fixed
    nodes); for the compliance with homogeneous Dirichlet data lam = T.
    """
    rho = np.asarray(rho, dtype=np.float64).ravel()
    rp = np.ones_like(rho)
    for _ in range(int(p) - 1):
        rp = rp * rho
    dk = p * rp * (kmax - kmin)
    K0 = element_stiffness(grid.hx, grid.hy, grid.hz)
    en = grid.element_nodes()
    Te = np.asarray(T).ravel()[en]
    le = np.asarray(lam).ravel()[en]
    q = np.einsum("ea,ab,eb->e", le, K0, Te)
    return -dk * q


def heat_source(rho, f0, p):
    """Section 2.1 eq. (material), second line: element heat generation
    f_e = f0 (1 - rho_e^p), rho^p by repeated products."""
    rho = np.asarray(rho, dtype=np.float64)
    rp = rho.copy()
    for _ in range(int(p) - 1):
        rp = rp * rho
    return f0 * (1.0 - rp)


def heat_source_load(grid, rho, f0, p):
    """Nodal load of the design-dependent source: f_n = sum_{e ni n} f0 (1 - rho_e^p) V / 8."""
    return element_load(grid, heat_source(np.asarray(rho).ravel(), f0, p))


def mean_temperature_weights(grid):
    """Section 2.3 eq. (cost function) on Q1 nodes: c = (1/|Omega|) int T dx = w^T T.

    The paper averages its cell temperatures; for the nodal Q1 field the same
    mean is the integral of T over the box divided by the box volume, whose
    weights are the consistent load of the constant source 1/|Omega|.
    """
    return element_load(grid, 1.0 / (grid.nelem * grid.vol))


def sensitivity_heat_source(grid, rho, T, lam, kmin, kmax, p, f0):
    """dc/drho_e = lam^T (df/drho_e - dA/drho_e T)  (section 2.3, with the
    design-dependent source of eq. (material)).

    df/drho_e puts -f0 p rho_e^(p-1) V / 8 on each node of e, so
    dc/drho_e = -(dk/drho)_e lam_e^T K0 T_e - f0 p rho_e^(p-1) (V / 8) sum_a lam_a.
    lam is the adjoint (zero on fixed nodes); T carries the fixed values.
    """
    rho = np.asarray(rho, dtype=np.float64).ravel()
    rp = np.ones_like(rho)
    for _ in range(int(p) - 1):
        rp = rp * rho
    en = grid.element_nodes()
    lsum = np.asarray(lam, dtype=np.float64).ravel()[en].sum(axis=1)
    return sensitivity(grid, rho, T, lam, kmin, kmax, p) - f0 * p * rp * (grid.vol / 8.0) * lsum


def apply_elementwise(grid, kelem, x, mask=None, zslab=16):
    """y = A x by element scatter, in z-slabs (bounded memory for large grids).

    With ``mask`` the masked form P A P x + (I - P) x is returned.
    """
    kelem = np.asarray(kelem, dtype=np.float64).reshape(grid.nz, grid.ny, grid.nx)
    x3 = np.asarray(x, dtype=np.float64).reshape(grid.nnz, grid.nny, grid.nnx)
    if mask is not None:
        m3 = np.asarray(mask).reshape(x3.shape).astype(bool)
        x3 = np.where(m3, 0.0, x3)
    K0 = element_stiffness(grid.hx, grid.hy, grid.hz)
    y3 = np.zeros_like(x3)
    for z0 in range(0, grid.nz, zslab):
        z1 = min(grid.nz, z0 + zslab)
        ks = kelem[z0:z1]
        xe = np.empty((z1 - z0, grid.ny, grid.nx, 8))
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            xe[..., a] = x3[z0 + az:z1 + az, ay:ay + grid.ny, ax:ax + grid.nx]
        ye = np.einsum("ab,zyxb->zyxa", K0, xe) * ks[..., None]
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            y3[z0 + az:z1 + az, ay:ay + grid.ny, ax:ax + grid.nx] += ye[..., a]
    if mask is not None:
        y3 = np.where(m3, np.asarray(x).reshape(y3.shape), y3)
    return y3.ravel()


class DiffOperator:
    """The masked operator y = P A P x + (I - P) x evaluated in difference form.

    For a free row n, (A x)_n = sum_{m != n} A_nm (x_m - x_n) because the rows
    of A (a sum of element matrices) sum to zero; fixed nodes enter with x = 0.
    This is the same matrix as ``masked_operator``; only the rounding differs:
    it stays proportional to the local variation of x instead of its size,
    which matters when T reaches ~1/k_min on low-conductivity islands.
    """

    def __init__(self, A, mask):
        coo = sp.coo_matrix(A)
        off = coo.row != coo.col
        self.r = coo.row[off]
        self.c = coo.col[off]
        self.v = coo.data[off]
        self.mask = np.asarray(mask).ravel().astype(bool)
        self.shape = A.shape

    def __matmul__(self, x):
        x = np.asarray(x, dtype=np.float64)
        xm = np.where(self.mask, 0.0, x)
        y = np.bincount(self.r, weights=self.v * (xm[self.c] - xm[self.r]), minlength=self.shape[0])
        return np.where(self.mask, x, y)

    def free_product(self, x):
        """(P A P x) on free rows, 0 on fixed rows, for x of any float precision:
        neighbour differences are formed in the precision of x, then rounded."""
        xm = np.where(self.mask, np.zeros((), dtype=x.dtype), x)
        d = (xm[self.c] - xm[self.r]).astype(np.float64)
        y = np.bincount(self.r, weights=self.v * d, minlength=self.shape[0])
        return np.where(self.mask, 0.0, y)


def relative_residual_diff(A, T, f, mask, td=None, T_lo=None):
    """||(f - A T)_F|| / ||b_F|| with A T evaluated in difference form (see DiffOperator).

    Fixed nodes carry their values ``td`` (zero when None) in T.  With T_lo the
    solution is T + T_lo (a double-binary64 value) and both parts are
    differenced separately.
    """
    mask = np.asarray(mask).ravel().astype(bool)
    T = np.asarray(T, dtype=np.float64).ravel()
    coo = sp.coo_matrix(A)
    off = coo.row != coo.col
    r, c, v = coo.row[off], coo.col[off], coo.data[off]
    d = T[c] - T[r]
    if T_lo is not None:
        Tl = np.asarray(T_lo, dtype=np.float64).ravel()
        d = d + (Tl[c] - Tl[r])
    AT = np.bincount(r, weights=v * d, minlength=A.shape[0])
    res = (np.asarray(f).ravel() - AT)[~mask]
    b = lifted_rhs(A, f, mask, td)[~mask]
    return float(np.linalg.norm(res) / np.linalg.norm(b))


def residual_rows(grid, rho, kmin, kmax, p, T, f_rows, nodes, T_lo=None):
    """Rows of f - A T at the given (free) nodes, one node at a time from the
    element matrices, in difference form: (A T)_n = sum over the elements e
    around n of k_e sum_b K0[a][b] (T_b - T_a), a = n's local index in e (rows
    of K0 sum to zero).  Needs only the densities and temperatures around the
    listed nodes, so it runs at any grid size.  Returns the rows and, for
    scaling round-off bounds, the sums of the absolute values of the terms.
    ``f_rows`` holds the load at the listed nodes.  Fixed nodes carry their
    values in T (zero for the model problem).
    """
    nodes = np.asarray(nodes, dtype=np.int64).ravel()
    T = np.asarray(T).reshape(-1)
    f_rows = np.asarray(f_rows, dtype=np.float64).reshape(-1)
    rho = np.asarray(rho).reshape(-1)
    Tl = None if T_lo is None else np.asarray(T_lo).reshape(-1)
    K0 = element_stiffness(grid.hx, grid.hy, grid.hz)
    i = nodes % grid.nnx
    j = (nodes // grid.nnx) % grid.nny
    k = nodes // (grid.nnx * grid.nny)

    def diff(ib, ia):
        # T_b - T_a with a double-binary64 T: both parts differenced separately
        d = T[ib].astype(np.float64) - T[ia].astype(np.float64)
        if Tl is not None:
            d = d + (Tl[ib].astype(np.float64) - Tl[ia].astype(np.float64))
        return d

    AT = np.zeros(nodes.size)
    absum = np.zeros(nodes.size)
    for c in range(8):  # element whose corner (c & 1, c >> 1 & 1, c >> 2 & 1) is away from n
        ex = i - 1 + (c & 1)
        ey = j - 1 + ((c >> 1) & 1)
        ez = k - 1 + ((c >> 2) & 1)
        ok = (ex >= 0) & (ex < grid.nx) & (ey >= 0) & (ey < grid.ny) & (ez >= 0) & (ez < grid.nz)
        exc, eyc, ezc = np.where(ok, ex, 0), np.where(ok, ey, 0), np.where(ok, ez, 0)
        ke = conductivity(rho[grid.element_index(exc, eyc, ezc)], kmin, kmax, p)
        a = np.where(ok, (i - exc) + 2 * (j - eyc) + 4 * (k - ezc), 0)
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            d = diff(grid.node_index(exc + bx, eyc + by, ezc + bz), nodes)
            term = np.where(ok, ke * K0[a, b] * d, 0.0)
            AT += term
            absum += np.abs(term)
    return f_rows - AT, absum


def relative_residual_slabs(grid, rho, kmin, kmax, p, T, f, mask, T_lo=None, zslab=8):
    """||(f - A T)_F|| / ||f_F|| for zero fixed values, with A T evaluated element
    by element in difference form (k_e K0 (T_b - T_a), hi and lo parts of a
    double-binary64 T differenced separately), z-slab by z-slab so that the
    memory stays bounded on grids too large to assemble.
    """
    K0 = element_stiffness(grid.hx, grid.hy, grid.hz)
    nz, ny, nx = grid.nz, grid.ny, grid.nx
    rho3 = np.asarray(rho).reshape(nz, ny, nx)
    T3 = np.asarray(T, dtype=np.float64).reshape(grid.nnz, grid.nny, grid.nnx)
    Tl3 = None if T_lo is None else np.asarray(T_lo, dtype=np.float64).reshape(T3.shape)
    AT = np.zeros(T3.shape)
    for z0 in range(0, nz, zslab):
        z1 = min(nz, z0 + zslab)
        ks = conductivity(rho3[z0:z1], kmin, kmax, p)
        corner = []
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            sl = (slice(z0 + az, z1 + az), slice(ay, ay + ny), slice(ax, ax + nx))
            corner.append((T3[sl], None if Tl3 is None else Tl3[sl]))
        for a in range(8):
            ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
            ya = np.zeros(ks.shape)
            for b in range(8):
                if b == a:
                    continue
                d = corner[b][0] - corner[a][0]
                if Tl3 is not None:
                    d = d + (corner[b][1] - corner[a][1])
                ya += K0[a, b] * d
            AT[z0 + az:z1 + az, ay:ay + ny, ax:ax + nx] += ks * ya
    free = ~np.asarray(mask).reshape(-1).astype(bool)
    res = (np.asarray(f, dtype=np.float64).reshape(-1) - AT.reshape(-1))[free]
    return float(np.linalg.norm(res) / np.linalg.norm(np.asarray(f, dtype=np.float64).reshape(-1)[free]))
