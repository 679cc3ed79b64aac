"""Memory layouts for the largest grids: the coarse-coarse set-up solved in
groups, FP32 storage of the density and the lean layout (basis master in the
PCG work vectors) compute exactly what the default layout computes."""
import numpy as np
import pytest
import torch

from gpu_common import KMAX, P, field, patch_mask, to_dev
from paper_2410_06850_amd._lib import MsmgError as L_ERR

pytestmark = pytest.mark.gpu

N, H, SD, KMIN = 32, 4, 2, 1e-6   # 8^3 coarse cells, 4^3 coarse-coarse cells


@pytest.fixture(scope="module")
def pkg():
    import paper_2410_06850_amd as p
    return p


def _setup(pkg, rho, **opts):
    # a fixed level-1 launch shape (the tuner picks one by timing; handles
    # with different shapes hold bases that differ in the last bits)
    s = pkg.Solver(N, H=H, sd=SD, autotune=0, **opts)
    s.setup(rho, KMIN, KMAX, P, to_dev(patch_mask(N), torch.uint8))
    return s


def test_grouped_cc_setup_matches_single_group(pkg):
    """Cells of a group stop when they converge, so the grouping does not change
    any cell's arithmetic: spectra, A_cc and the preconditioner agree bitwise."""
    print("case cc groups of 5 vs one group, 32^3 grf contrast 1e6", flush=True)
    rho = to_dev(field(N, "grf", 5))
    a = _setup(pkg, rho)
    b = _setup(pkg, rho, cc_group=5)
    n_cc = (N // H // SD) ** 3 * 17
    assert torch.equal(a.export(3, n_cc), b.export(3, n_cc))
    assert torch.equal(a.export(4, n_cc * n_cc), b.export(4, n_cc * n_cc))
    r = torch.randn(a.nnodes, dtype=torch.float64, generator=torch.Generator().manual_seed(3)).to("cuda")
    assert torch.equal(a.precondition(r), b.precondition(r))


def test_lean_layout_and_fp32_density_match_default(pkg):
    """F32 densities stored as F32 (lean layout) or upcast to F64 (default
    layout) define the same operator: same basis, iterations and solution."""
    print("case lean + FP32 density storage vs default, 32^3 grf contrast 1e6", flush=True)
    rho32 = to_dev(field(N, "grf", 6), torch.float32)
    a = _setup(pkg, rho32)
    b = _setup(pkg, rho32, rho_storage=1, lean_memory=1)
    nb = a.nnodes * 4
    assert torch.equal(a.export(1, nb), b.export(1, nb))
    f = torch.ones(a.nnodes, dtype=torch.float64, device="cuda") / N ** 3
    Ta, ia = a.solve(f, rtol=1e-8)
    Tb, ib = b.solve(f, rtol=1e-8)
    assert ia.code == 0 and ib.iterations == ia.iterations
    assert torch.equal(Ta, Tb)
    # the lean layout keeps neither the basis after a solve nor a copy of A_cc
    with pytest.raises(L_ERR):
        b.export(1, nb)
    n_cc = (N // H // SD) ** 3 * 17
    with pytest.raises(L_ERR):
        b.export(4, n_cc * n_cc)
    # F32 storage refuses F64 densities
    with pytest.raises(L_ERR):
        b.setup(rho32.double(), KMIN, KMAX, P, to_dev(patch_mask(N), torch.uint8))
