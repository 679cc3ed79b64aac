"""Oracle, part 2: the three-grid multiscale multigrid preconditioner and PCG.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (section 3):
  * three nested spaces W_cc in W_c in W_h; R_c rows are local eigenvectors of
    eq. (spepb) on every coarse element, R_cc rows are eigenvectors of
    eq. (spectral cc) on every coarse-coarse element expressed in the W_c basis;
  * Galerkin coarse operators A_c = R_c A R_c^T and A_cc = R_cc A_c R_cc^T;
  * the right-hand operator of both spectral problems is diagonal, and with
    eigenvectors normalised in that form the coarse-coarse problem becomes a
    standard eigenproblem;
  * one preconditioner application is Algorithm 1 (pre-smooth, restrict,
    coarse pre-smooth, restrict, direct coarse-coarse solve, prolong, coarse
    post-smooth, prolong, post-smooth), used inside CG (section 4).

Readings taken where the paper is silent or written for cell-centred unknowns
(each is also listed in the design notes):
  * nodal ownership: along each axis nodes 0..N are cut into runs of H nodes,
    the last run keeps the remainder (H + 1 nodes when H divides N); a coarse
    cell owns the box product of its runs, so every node has one owner and the
    local spaces are disjoint;
  * local stiffness = sum of k_e K0 over elements whose 8 nodes are all owned
    by the cell (the analogue of "internal faces"), on owned free nodes;
  * local right-hand form = k-weighted lumped mass over the same elements
    (diagonal, as the paper requires);
  * coarse-coarse cells group sd^3 coarse cells (remainders join the last
    group); their stiffness keeps elements whose nodes all belong to the group,
    and the right-hand form is the identity (the normalised-basis reading);
  * fixed-temperature nodes are removed from every space;
  * the coarse-coarse "correction e_cc <- A_cc r_cc" is read as the direct
    solve A_cc e_cc = r_cc (its comment names a direct solver);
  * smoothers: level 0 Chebyshev-Jacobi of a given degree on D^-1 A over
    [lo, hi]; level 1 one forward (pre) / backward (post) sweep of block
    Gauss-Seidel over the 8 parity colours of the coarse cells;
  * CG uses the Polak-Ribiere (flexible) beta and stops on the true relative
    residual ||b - A x|| / ||b||;
  * fine-level products with A are evaluated in difference form (same matrix,
    rounding that does not grow with the size of T; see q1.DiffOperator).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import q1


@dataclasses.dataclass
class Options:
    H: int = 8            # coarse cell size in elements per axis
    sd: int = 8           # coarse cells per coarse-coarse cell per axis
    Lc: int = 4           # eigenvectors kept per coarse cell
    Lcc: int = 17         # eigenvectors kept per coarse-coarse cell
    cheb_degree: int = 2  # level-0 Chebyshev degree (number of smoothing steps)
    cheb_lo: float = 0.15
    cheb_hi: float = 1.5
    # adaptive local basis (section 3 allows a count l_c^i per coarse cell):
    # when > 0, cell i keeps its eigenpairs with lambda <= lc_threshold *
    # lambda_ref (at least one, at most Lc), lambda_ref = (pi / (H h_max))^2
    # the first Neumann eigenvalue of a homogeneous cube of the cell's size
    lc_threshold: float = 0.0


def axis_runs(n_elems, H):
    """Node runs along one axis: [(start, end_exclusive)] over nodes 0..n_elems."""
    nc = n_elems // H
    if nc < 1 or H < 2:
        raise ValueError("need H >= 2 and at least H elements per axis")
    starts = [c * H for c in range(nc)]
    ends = starts[1:] + [n_elems + 1]
    return list(zip(starts, ends))


def axis_groups(nc, sd):
    """Coarse-cell groups along one axis: [(start, end_exclusive)] over 0..nc."""
    ng = max(1, nc // sd)
    starts = [g * sd for g in range(ng)]
    ends = starts[1:] + [nc]
    return list(zip(starts, ends))


def _fix_sign(phi, m):
    """Sign convention: sum_n m_n phi_n > 0, else the first largest-|.| entry > 0.

    Only cosmetic: every quantity the preconditioner produces is invariant under
    a sign (or any orthogonal change) of the basis of one local space.
    """
    s = float(m @ phi)
    if abs(s) > 1e-8 * np.sqrt(float(m.sum())):
        return phi if s > 0 else -phi
    a = np.abs(phi)
    idx = int(np.flatnonzero(a >= (1.0 - 1e-8) * a.max())[0])
    return phi if phi[idx] > 0 else -phi


class Hierarchy:
    """Coarse spaces, Galerkin operators and the factorised coarse-coarse matrix.

    Built from scratch for one density field (the paper's flowchart rebuilds
    the preconditioner whenever the design changes).
    """

    def __init__(self, grid, rho, kmin, kmax, p, mask, opts=None, keep_local=True):
        self.g = grid
        self.o = opts or Options()
        self.kmin, self.kmax, self.p = kmin, kmax, p
        self.n_unknowns = grid.nnodes
        self.mask = np.asarray(mask).ravel().astype(bool)
        self.k = q1.conductivity(np.asarray(rho).ravel(), kmin, kmax, p)
        A = q1.assemble(grid, self.k)
        self.A_csr = q1.masked_operator(A, self.mask)      # Galerkin products
        self.A = q1.DiffOperator(A, self.mask)             # fine-level products
        self.diag = self.A_csr.diagonal().copy()
        self._partition()
        self._level1(keep_local)
        self._level2()

    # -- partition ---------------------------------------------------------
    def _axis_runs(self, axis):
        """Runs of unknowns along one axis (nodes here)."""
        return axis_runs((self.g.nx, self.g.ny, self.g.nz)[axis], self.o.H)

    def _axis_unknowns(self):
        return (self.g.nnx, self.g.nny, self.g.nnz)

    def unknown_index(self, i, j, k):
        return self.g.node_index(i, j, k)

    def _partition(self):
        g, o = self.g, self.o
        self.runs = [self._axis_runs(0), self._axis_runs(1), self._axis_runs(2)]
        self.nc = [len(r) for r in self.runs]
        self.groups = [axis_groups(n, o.sd) for n in self.nc]
        self.ncc = [len(gr) for gr in self.groups]
        ncx, ncy, ncz = self.nc
        self.cells = []  # (cx, cy, cz) in x-fastest order
        for cz in range(ncz):
            for cy in range(ncy):
                for cx in range(ncx):
                    self.cells.append((cx, cy, cz))
        # owner coarse cell of every node, per axis
        self.own_axis = []
        for ax, n in enumerate(self._axis_unknowns()):
            o_ax = np.empty(n, dtype=np.int64)
            for c, (s, e) in enumerate(self.runs[ax]):
                o_ax[s:e] = c
            self.own_axis.append(o_ax)
        self.grp_axis = []
        for ax in range(3):
            gr = np.empty(self.nc[ax], dtype=np.int64)
            for j, (s, e) in enumerate(self.groups[ax]):
                gr[s:e] = j
            self.grp_axis.append(gr)

    def cell_id(self, cx, cy, cz):
        return (cz * self.nc[1] + cy) * self.nc[0] + cx

    def colour(self, cx, cy, cz):
        return (cx % 2) + 2 * (cy % 2) + 4 * (cz % 2)

    def cell_nodes(self, cx, cy, cz):
        """Owned global node ids of a coarse cell, local x-fastest order."""
        (sx, ex), (sy, ey), (sz, ez) = self.runs[0][cx], self.runs[1][cy], self.runs[2][cz]
        kk, jj, ii = np.meshgrid(np.arange(sz, ez), np.arange(sy, ey), np.arange(sx, ex),
                                 indexing="ij")
        return self.unknown_index(ii.ravel(), jj.ravel(), kk.ravel())

    def _box_elements(self, xr, yr, zr):
        """Elements whose 8 nodes lie in the node box xr * yr * zr (half-open ranges)."""
        g = self.g
        kk, jj, ii = np.meshgrid(np.arange(zr[0], zr[1] - 1), np.arange(yr[0], yr[1] - 1),
                                 np.arange(xr[0], xr[1] - 1), indexing="ij")
        return g.element_index(ii.ravel(), jj.ravel(), kk.ravel())

    # -- level 1: eq. (spepb) ---------------------------------------------
    def local_problem(self, cx, cy, cz):
        """Local Neumann stiffness, lumped k-weighted mass and node ids (free nodes only)."""
        g = self.g
        nodes = self.cell_nodes(cx, cy, cz)
        xr, yr, zr = self.runs[0][cx], self.runs[1][cy], self.runs[2][cz]
        elems = self._box_elements(xr, yr, zr)
        K0 = q1.element_stiffness(g.hx, g.hy, g.hz)
        nl = len(nodes)
        K = np.zeros((nl, nl))
        m = np.zeros(nl)
        if len(elems):
            en = g.element_nodes(elems)
            # global node (i, j, k) -> local x-fastest index inside the owned box
            gi = en % g.nnx
            gj = (en // g.nnx) % g.nny
            gk = en // (g.nnx * g.nny)
            lx, ly = xr[1] - xr[0], yr[1] - yr[0]
            li = (gi - xr[0]) + lx * ((gj - yr[0]) + ly * (gk - zr[0]))
            ke = self.k[elems]
            for a in range(8):
                np.add.at(m, li[:, a], ke * g.vol / 8.0)
                for b in range(8):
                    np.add.at(K, (li[:, a], li[:, b]), ke * K0[a, b])
        free = ~self.mask[nodes]
        return K[np.ix_(free, free)], m[free], nodes[free]

    def _level1(self, keep_local):
        o = self.o
        rows, cols, vals = [], [], []
        self.cell_rows = []      # coarse dof ids of each cell
        self.cell_evals = []     # local eigenvalues of each cell
        self.cell_gaps = []      # lambda_L - lambda_{L-1} (inf when the space is full)
        self.cell_basis = []     # (node ids, Phi) per cell when keep_local
        self.cell_mass = []
        r = 0
        theta = o.lc_threshold * self.lambda_ref() if o.lc_threshold > 0 else None
        for (cx, cy, cz) in self.cells:
            K, m, nodes = self.local_problem(cx, cy, cz)
            nl = min(o.Lc, len(nodes))
            if theta is not None and nl > 1:
                # the count of eigenvalues at or below the threshold (at least one)
                lam_all = sla.eigh(K, np.diag(m), eigvals_only=True, subset_by_index=[0, nl - 1], driver="gvx")
                nl = max(1, int(np.count_nonzero(lam_all <= theta)))
            ids = list(range(r, r + nl))
            self.cell_rows.append(np.array(ids, dtype=np.int64))
            if nl == 0:
                self.cell_evals.append(np.zeros(0))
                if keep_local:
                    self.cell_basis.append((nodes, np.zeros((len(nodes), 0))))
                    self.cell_mass.append(m)
                continue
            top = min(nl, len(nodes) - 1)  # one eigenvalue past the cut (gap diagnostic)
            lam, phi = sla.eigh(K, np.diag(m), subset_by_index=[0, top], driver="gvx")
            self.cell_gaps.append(lam[nl] - lam[nl - 1] if top == nl else np.inf)
            lam, phi = lam[:nl], phi[:, :nl]
            for j in range(nl):
                phi[:, j] = _fix_sign(phi[:, j], m)
            self.cell_evals.append(lam)
            if keep_local:
                self.cell_basis.append((nodes, phi))
                self.cell_mass.append(m)
            for j in range(nl):
                rows.append(np.full(len(nodes), r + j))
                cols.append(nodes)
                vals.append(phi[:, j])
            r += nl
        self.n_c = r
        self.Rc = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(self.n_c, self.n_unknowns)).tocsr()
        self.level1_operators()

    def lambda_ref(self):
        """(pi / (H h_max))^2: the first nonzero Neumann eigenvalue of a
        homogeneous cube with the coarse cell's nominal side, the scale of the
        adaptive threshold."""
        hmax = max(self.g.hx, self.g.hy, self.g.hz)
        return (np.pi / (self.o.H * hmax)) ** 2

    def level1_operators(self):
        """A_c = R_c A R_c^T, its diagonal-block inverses and the colour classes."""
        self.Ac = sp.csr_matrix(self.Rc @ self.A_csr @ self.Rc.T)
        # block-diagonal inverse and colour classes for block Gauss-Seidel
        self.colour_rows = [[] for _ in range(8)]
        inv_blocks = []
        Acd = self.Ac.tocsr()
        for ci, (cx, cy, cz) in enumerate(self.cells):
            ids = self.cell_rows[ci]
            if len(ids) == 0:
                continue
            self.colour_rows[self.colour(cx, cy, cz)].append(ids)
            blk = Acd[ids][:, ids].toarray()
            inv_blocks.append((ids, np.linalg.inv(blk)))
        self.colour_rows = [np.concatenate(c) if c else np.zeros(0, dtype=np.int64)
                            for c in self.colour_rows]
        ri, ci_, vi = [], [], []
        for ids, inv in inv_blocks:
            ri.append(np.repeat(ids, len(ids)))
            ci_.append(np.tile(ids, len(ids)))
            vi.append(inv.ravel())
        self.Dc_inv = sp.coo_matrix((np.concatenate(vi), (np.concatenate(ri), np.concatenate(ci_))),
                                    shape=(self.n_c, self.n_c)).tocsr()
        self._gs_parts = []
        for c in range(8):
            rr = self.colour_rows[c]
            self._gs_parts.append((rr, Acd[rr], self.Dc_inv[rr][:, rr]))

    # -- level 2: eq. (spectral cc) -----------------------------------------
    def cc_elements_mask(self):
        """Elements whose 8 nodes belong to coarse cells of one coarse-coarse cell."""
        g = self.g
        ex, ey, ez = g.element_coords()
        ok = np.ones(g.nelem, dtype=bool)
        for ax, e in enumerate((ex, ey, ez)):
            ga = self.grp_axis[ax][self.own_axis[ax][e]]
            gb = self.grp_axis[ax][self.own_axis[ax][e + 1]]
            ok &= ga == gb
        return ok

    def cc_stiffness(self):
        """Stiffness of the elements inside one coarse-coarse cell, masked."""
        elems = np.flatnonzero(self.cc_elements_mask())
        return q1.masked_operator(q1.assemble(self.g, self.k, elems), self.mask)

    def _level2(self):
        o = self.o
        Kcc = self.cc_stiffness()
        # the identity part of the masked form never meets R_c (zero on fixed nodes)
        KR = (self.Rc @ Kcc @ self.Rc.T).tocsr()
        ncx, ncy, ncz = self.ncc
        cc_members = {}
        for ci, (cx, cy, cz) in enumerate(self.cells):
            key = (self.grp_axis[0][cx], self.grp_axis[1][cy], self.grp_axis[2][cz])
            cc_members.setdefault(key, []).append(ci)
        rows, cols, vals = [], [], []
        self.cc_rows, self.cc_evals, self.cc_dofs = [], [], []
        self.cc_gaps, self.cc_norms = [], []
        r = 0
        for jz in range(ncz):
            for jy in range(ncy):
                for jx in range(ncx):
                    members = cc_members[(jx, jy, jz)]
                    dofs = np.concatenate([self.cell_rows[c] for c in members])
                    self.cc_dofs.append(dofs)
                    nl = min(o.Lcc, len(dofs))
                    if nl == 0:
                        self.cc_rows.append(np.zeros(0, dtype=np.int64))
                        self.cc_evals.append(np.zeros(0))
                        continue
                    G = KR[dofs][:, dofs].toarray()
                    G = 0.5 * (G + G.T)
                    top = min(nl, len(dofs) - 1)
                    lam, v = sla.eigh(G, subset_by_index=[0, top], driver="evx")
                    self.cc_gaps.append(lam[nl] - lam[nl - 1] if top == nl else np.inf)
                    self.cc_norms.append(float(np.abs(G).sum(axis=1).max()))
                    lam, v = lam[:nl], v[:, :nl]
                    one = np.ones(len(dofs))
                    for j in range(nl):
                        v[:, j] = _fix_sign(v[:, j], one)
                    self.cc_rows.append(np.arange(r, r + nl))
                    self.cc_evals.append(lam)
                    for j in range(nl):
                        rows.append(np.full(len(dofs), r + j))
                        cols.append(dofs)
                        vals.append(v[:, j])
                    r += nl
        self.n_cc = r
        self.Rcc = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(self.n_cc, self.n_c)).tocsr()
        self.level2_operators()

    def level2_operators(self):
        """A_cc = R_cc A_c R_cc^T and its Cholesky factor."""
        self.Acc = (self.Rcc @ self.Ac @ self.Rcc.T).toarray()
        self.Acc = 0.5 * (self.Acc + self.Acc.T)
        self.Acc_chol = sla.cho_factor(self.Acc, lower=True)

    # -- smoothers ------------------------------------------------------------
    def chebyshev(self, r):
        """Level-0 smoother S^-1 r: Chebyshev iteration on D^-1 A from a zero guess.

        Textbook three-term Chebyshev acceleration for the interval [lo, hi] of
        the spectrum of D^-1 A (e.g. Saad, Iterative Methods for Sparse Linear
        Systems, 2nd ed., Alg. 12.1); ``degree`` steps cost degree - 1 products
        with A.  The error after the steps is T_d((theta - lam)/delta) /
        T_d(theta/delta) times the initial error on each eigenmode lam.
        """
        o = self.o
        theta = 0.5 * (o.cheb_hi + o.cheb_lo)
        delta = 0.5 * (o.cheb_hi - o.cheb_lo)
        sigma = theta / delta
        rho_prev = 1.0 / sigma
        d = (r / self.diag) / theta
        x = d.copy()
        for _ in range(1, o.cheb_degree):
            res = r - self.A @ x
            rho = 1.0 / (2.0 * sigma - rho_prev)
            d = rho * rho_prev * d + (2.0 * rho / delta) * (res / self.diag)
            x = x + d
            rho_prev = rho
        return x

    def gs_forward(self, b):
        """S_c^-1 b: one block Gauss-Seidel sweep, colours 0..7, zero initial guess."""
        x = np.zeros(self.n_c)
        for c in range(8):
            rr, Arows, Dinv = self._gs_parts[c]
            if len(rr) == 0:
                continue
            x[rr] += Dinv @ (b[rr] - Arows @ x)
        return x

    def gs_backward(self, b):
        """S_c^-T b: the transposed sweep, colours 7..0, zero initial guess."""
        x = np.zeros(self.n_c)
        for c in range(7, -1, -1):
            rr, Arows, Dinv = self._gs_parts[c]
            if len(rr) == 0:
                continue
            x[rr] += Dinv @ (b[rr] - Arows @ x)
        return x

    # -- Algorithm 1 --------------------------------------------------------------
    def precondition(self, r0):
        """One three-grid iteration (Algorithm 1) applied to a residual r0."""
        r0 = np.asarray(r0, dtype=np.float64).copy()
        r0[self.mask] = 0.0
        r1 = self.chebyshev(r0)                                  # pre-smoothing
        rc = self.Rc @ (r0 - self.A @ r1)                        # restriction
        rc0 = self.gs_forward(rc)                                # coarse pre-smoothing
        rcc = self.Rcc @ (rc - self.Ac @ rc0)                    # restriction
        ecc = sla.cho_solve(self.Acc_chol, rcc)                  # direct coarse-coarse solve
        rc1 = rc0 + self.Rcc.T @ ecc                             # prolongation
        ec = rc1 + self.gs_backward(rc - self.Ac @ rc1)          # coarse post-smoothing
        r2 = r1 + self.Rc.T @ ec                                 # prolongation
        return r2 + self.chebyshev(r0 - self.A @ r2)             # post-smoothing


@dataclasses.dataclass
class PCGResult:
    x: np.ndarray           # iterate rounded to binary64
    iterations: int
    rel_res: float          # true relative residual at exit
    status: str             # "converged" | "maxit" | "breakdown"
    history: list
    x_lo: np.ndarray = None  # x_ext - x (the part binary64 cannot hold)


def pcg(A, b, precond, x0=None, rtol=1e-8, maxit=1000, mask=None):
    """Preconditioned CG with the Polak-Ribiere beta z_{k+1}^T (r_{k+1} - r_k) / z_k^T r_k.

    Stops when the recursive relative residual reaches ``rtol`` and the true
    residual ||b - A x|| / ||b|| confirms it; if it does not, the residual is
    replaced by the true one and the search direction restarts from z.
    Vectors live on all nodes; entries on fixed nodes stay zero.  The iterate
    x is accumulated in extended precision (np.longdouble) and the true
    residual is formed from its neighbour differences: at high conductivity
    contrast T is ~1/k_min on islands and a binary64 iterate alone cannot
    reach relative residuals near 1e-8 (A must be a DiffOperator).
    """
    ext = np.longdouble
    b = np.asarray(b, dtype=np.float64)
    fr = np.ones(len(b), dtype=bool) if mask is None else ~np.asarray(mask).ravel().astype(bool)
    bb = np.where(fr, b, 0.0)
    nb = np.linalg.norm(bb)

    def true_res(xe):
        return bb - A.free_product(xe)

    def out(xe, it, rel, st, hist):
        x64 = xe.astype(np.float64)
        return PCGResult(x64, it, rel, st, hist, (xe - x64).astype(np.float64))

    x = np.zeros(len(b), dtype=ext) if x0 is None else np.where(fr, np.asarray(x0, dtype=np.float64), 0.0).astype(ext)
    r = true_res(x)
    hist = [np.linalg.norm(r) / nb]
    if hist[0] <= rtol:
        return out(x, 0, hist[0], "converged", hist)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    for it in range(1, maxit + 1):
        q = np.where(fr, A @ p, 0.0)
        pq = float(p @ q)
        if not (pq > 0.0) or not (rz > 0.0):
            return out(x, it - 1, float(np.linalg.norm(true_res(x)) / nb), "breakdown", hist)
        alpha = rz / pq
        x = x + ext(alpha) * p.astype(ext)
        r_new = r - alpha * q
        rel = np.linalg.norm(r_new) / nb
        hist.append(rel)
        restart = False
        if rel <= rtol:
            true_r = true_res(x)
            true_rel = np.linalg.norm(true_r) / nb
            if true_rel <= rtol:
                return out(x, it, float(true_rel), "converged", hist)
            r_new = true_r
            restart = True
        z = precond(r_new)
        if restart:
            beta = 0.0
        else:
            beta = float(z @ (r_new - r)) / rz
        rz = float(z @ r_new)
        p = z + beta * p
        r = r_new
    return out(x, maxit, float(np.linalg.norm(true_res(x)) / nb), "maxit", hist)


def solve(grid, rho, f, mask, kmin, kmax, p, opts=None, rtol=1e-8, maxit=1000, td=None,
          x0=None, hier=None):
    """T from PCG-MsMG on the lifted system; returns (T, PCGResult, Hierarchy)."""
    h = hier or Hierarchy(grid, rho, kmin, kmax, p, mask, opts)
    Araw = q1.assemble(grid, h.k)
    b = q1.lifted_rhs(Araw, f, h.mask, td)
    bfree = np.where(h.mask, 0.0, b)
    res = pcg(h.A, bfree, h.precondition, x0=x0, rtol=rtol, maxit=maxit, mask=h.mask)
    T = res.x.copy()
    T[h.mask] = b[h.mask]
    res.x_lo[h.mask] = 0.0
    return T, res, h
