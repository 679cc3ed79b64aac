"""P2 certificates at the benchmark's own sizes: the oracle recomputes the true
relative residual of the GPU solution T + T_lo with its own element-by-element
operator (difference form, slab by slab) and requires <= rtol (1 + 1e-3).

256^3 is the benchmark configuration (GRF ell 16, seed 0, contrast 1e6, H 8,
sd 8, the mixed (BF16 k, FP32 R_c), FP64 and BF16-copies paths as bench.py runs
them); 512^3 uses the interpolation workload's field (GRF ell 32).  The four
cases take about 60 s.
"""
import pytest
import torch

import synth
from oracle import q1

pytestmark = pytest.mark.gpu

RTOL, KMIN, KMAX, P = 1e-8, 1e-6, 1.0, 3
PATHS = {"mixed": dict(vcycle_dtype=0, rho_v_dtype=2, basis_dtype=1), "fp64": {},
         "bf16": dict(vcycle_dtype=0, rho_v_dtype=2, basis_dtype=2)}


def _certify(n, ell, path):
    import paper_2410_06850_amd as pkg

    rho = synth.grf_rho(n, ell, seed=0).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    s = pkg.Solver(n, H=8, sd=8, **PATHS[path])
    s.setup(torch.from_numpy(rho).cuda(), KMIN, KMAX, P, torch.from_numpy(mask).cuda())
    f = s.element_load(const=1.0)
    T_lo = torch.empty_like(f)
    T, info = s.solve(f, rtol=RTOL, maxit=2000, T_lo=T_lo)
    print(f"  iterations {info.iterations} rel_res {info.rel_res:.3e}", flush=True)
    assert info.code == 0
    g = q1.Grid(n)
    f_or = q1.element_load(g, 1.0)
    cert = q1.relative_residual_slabs(g, rho, KMIN, KMAX, P, T.cpu().numpy(), f_or, mask, T_lo=T_lo.cpu().numpy())
    print(f"  oracle residual {cert:.3e}", flush=True)
    assert cert <= RTOL * (1 + 1e-3)


@pytest.mark.parametrize("path", list(PATHS))
def test_certificate_cube256_benchmark_config(path):
    print(f"case certificate cube256_grf16_c1e6 {path}", flush=True)
    _certify(256, 16, path)


def test_certificate_cube512_grf32_mixed():
    print("case certificate cube512_grf32_c1e6 mixed", flush=True)
    _certify(512, 32, "mixed")
