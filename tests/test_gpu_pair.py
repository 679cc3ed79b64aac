"""The batched state/adjoint pair (msmg_solve_pair): the paper's LS1 and LS2
of one set-up (section 4; section 2.3 eq. adjoint) advanced together, every
coefficient-reading kernel run once for both right-hand sides.

Each side runs the single-side PCG's arithmetic in the same order (the two
sides' workgroups only share the coefficient reads), so the pair must equal
two separate solves bitwise, with the same iteration counts; against the
oracle's direct state and adjoint solutions it holds the single solves'
1e-10 (noise fields) and 1e-8 (contrast 1e4)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from gpu_common import KMAX, P, field, patch_mask, rel, to_dev  # noqa: E402
from oracle import q1  # noqa: E402

pytestmark = pytest.mark.gpu

TD, F0 = 100.0, 1.0
MIXED = dict(vcycle_dtype=0, rho_v_dtype=2, basis_dtype=1)


def _oracle_pair(g, rho, mask, kmin):
    td = np.where(mask.astype(bool), TD, 0.0)
    A = q1.assemble(g, q1.conductivity(rho, kmin, KMAX, P))
    f = q1.heat_source_load(g, rho, F0, P)
    T = q1.solve_direct(A, f, mask, td)
    u = q1.adjoint_solve(A, q1.mean_temperature_weights(g), mask)
    return td, T, u


@pytest.mark.parametrize("n,kind,kmin,H,sd,opts,tol", [
    (16, "noise", 1e-3, 8, 2, {}, 1e-10),
    (16, "grf", 1e-4, 4, 2, {}, 1e-8),
    (16, "grf", 1e-4, 4, 2, MIXED, 1e-8),
    (24, "grf", 1e-4, 4, 3, dict(coarse_fused=0), 1e-8),
])
def test_pair_equals_two_solves_and_oracle(n, kind, kmin, H, sd, opts, tol):
    import paper_2410_06850_amd as pkg

    print(f"case pair cube{n}_{kind} kmin={kmin} H={H} opts={opts}", flush=True)
    rho = field(n, kind, 3)
    mask = patch_mask(n)
    g = q1.Grid(n)
    td, T_or, u_or = _oracle_pair(g, rho, mask, kmin)
    s = pkg.Solver(n, H=H, sd=sd, pair_rhs=1, **opts)
    s.setup(to_dev(rho), kmin, KMAX, P, to_dev(mask, torch.uint8), to_dev(td))
    f = s.heat_source_load(F0)
    w = s.mean_temperature_weights()
    T1, i1 = s.solve(f, rtol=1e-12, maxit=1000)
    u1, j1 = s.solve_adjoint(w, rtol=1e-12, maxit=1000)
    T2, u2, i2, j2 = s.solve_pair(f, w, rtol=1e-12, maxit=1000)
    print(f"  single it {i1.iterations}/{j1.iterations}, pair it {i2.iterations}/{j2.iterations}; "
          f"err T {rel(T2.cpu().numpy(), T_or):.2e} u {rel(u2.cpu().numpy(), u_or):.2e}", flush=True)
    assert i2.code == 0 and j2.code == 0
    assert (i2.iterations, j2.iterations) == (i1.iterations, j1.iterations)
    assert torch.equal(T1, T2) and torch.equal(u1, u2)
    assert rel(T2.cpu().numpy(), T_or) <= tol and rel(u2.cpu().numpy(), u_or) <= tol


def test_pair_at_the_shipped_hierarchy():
    """64^3 GRF at contrast 1e6 (H 8, sd 8, one coarse-coarse cell of
    dimension 2048), default mixed path, rtol 1e-8: the pair equals the two
    single solves bitwise; the sides stop at different iterations."""
    import paper_2410_06850_amd as pkg

    n = 64
    print("case pair cube64_grf4_c1e6 mixed", flush=True)
    rho = synth.grf_rho(n, 4, seed=0).ravel()
    mask = patch_mask(n)
    td = np.where(mask.astype(bool), TD, 0.0)
    s = pkg.Solver(n, H=8, sd=8, pair_rhs=1, **MIXED)
    s.setup(to_dev(rho), 1e-6, KMAX, P, to_dev(mask, torch.uint8), to_dev(td))
    f = s.heat_source_load(F0)
    w = s.mean_temperature_weights()
    T1, i1 = s.solve(f, rtol=1e-8, maxit=2000)
    u1, j1 = s.solve_adjoint(w, rtol=1e-8, maxit=2000)
    T2, u2, i2, j2 = s.solve_pair(f, w, rtol=1e-8, maxit=2000)
    print(f"  single it {i1.iterations}/{j1.iterations} ({i1.solve_ms + j1.solve_ms:.1f} ms), "
          f"pair it {i2.iterations}/{j2.iterations} ({i2.solve_ms:.1f} ms)", flush=True)
    assert i2.code == 0 and j2.code == 0
    assert (i2.iterations, j2.iterations) == (i1.iterations, j1.iterations)
    assert i1.iterations != j1.iterations
    assert torch.equal(T1, T2) and torch.equal(u1, u2)


def test_pair_needs_the_second_vector_set():
    import paper_2410_06850_amd as pkg
    from paper_2410_06850_amd import _lib as L

    s = pkg.Solver(16, H=8, sd=2)
    mask = patch_mask(16)
    s.setup(to_dev(field(16, "noise", 0)), 1e-3, KMAX, P, to_dev(mask, torch.uint8))
    f = s.element_load(const=1.0)
    with pytest.raises(L.MsmgError) as e:
        s.solve_pair(f, f.clone())
    assert e.value.code == L.MSMG_ESTATE
