"""TPFA parity at the shipped hierarchy: coarse cells of H = 8 cells, sd = 8
coarse cells per coarse-coarse cell, L_c = 4, L_cc = 17 (section 3, eq. spepb
and eq. spectral cc; Algorithm 1) on 64^3 cells: one coarse-coarse cell of
dimension 2048, sixteen 128-column pivot blocks of the batched Gauss-Jordan
inverse.

The oracle values come from tests/golden/tpfa_hierarchy.json, written by
tests/golden/make_tpfa_golden.py from the oracle alone.  Compared here: the
coarse-coarse eigenvalues, the spectra of A_cc and A_c, one preconditioner
application z = M^-1 r (norm, projection, 512 sampled cells; to 1e-10 or 100 x
the subspace error bound residual / gap), and PCG iterations to 1e-8 with
T_D = 100 and the paper's source within +-1 of the oracle's count.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from gpu_common import KMAX, P, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tpfa_hierarchy.json")
with open(GOLD_PATH) as _fh:
    GOLD = json.load(_fh)

_cache = {}


def _solver(name):
    import paper_2410_06850_amd as pkg

    if name in _cache:
        return _cache[name]
    c = GOLD[name]["case"]
    n = c["n"]
    rho = (synth.uniform_noise_rho(n, c["seed"]) if c["kind"] == "noise"
           else synth.grf_rho(n, c["ell"], seed=c["seed"])).ravel()
    flags = synth.dirichlet_patch_faces(n, n, n).ravel()
    s = pkg.Solver(n, discretisation="tpfa", H=8, sd=8, Lc=4, Lcc=17)
    td = torch.full((n ** 3,), GOLD[name]["pcg"]["td"], dtype=torch.float64, device="cuda")
    s.setup(to_dev(rho), c["kmin"], KMAX, P, to_dev(flags, torch.uint8), td)
    _cache.clear()  # one handle alive at a time
    _cache[name] = (s, n, rho)
    return _cache[name]


@pytest.mark.parametrize("name", list(GOLD))
def test_tpfa_production_spectra_match_oracle(name):
    print(f"case tpfa production spectra {name}", flush=True)
    gold = GOLD[name]
    s, n, rho = _solver(name)
    plan = s.plan()
    assert plan.n_cc == gold["n_cc"] and plan.ncells * 4 == gold["n_c"]
    st = s.export(5, plan.ncells, torch.int32).numpy()
    assert not np.any((st >> 28) & 1), "a level-1 cell did not converge"
    cc = s.export(3, plan.n_cc).numpy()
    want = np.array(gold["cc_evals"])
    err = np.abs(cc - want).max() / np.abs(want).max()
    print(f"  cc eigenvalues: max rel err {err:.2e}")
    assert err <= 1e-8
    Acc = s.export(4, plan.n_cc * plan.n_cc).numpy().reshape(plan.n_cc, plan.n_cc)
    ea = np.linalg.eigvalsh(0.5 * (Acc + Acc.T))
    want = np.array(gold["acc_evals"])
    err = np.abs(ea - want).max() / np.abs(want).max()
    bound = max(1e-8, 100 * gold["subspace_error_bound"])
    print(f"  A_cc spectrum: max rel err {err:.2e} (subspace bound {bound:.2e})")
    assert err <= bound
    L, ncx = 4, n // 8
    Ac = s.export(2, plan.ncells * 27 * L * L).numpy().reshape(plan.ncells, 27, L, L)
    D = np.zeros((plan.ncells * L, plan.ncells * L))
    for ci in range(plan.ncells):
        cx, cy, cz = ci % ncx, (ci // ncx) % ncx, ci // (ncx * ncx)
        for b in range(27):
            x, y, z = cx + b % 3 - 1, cy + (b // 3) % 3 - 1, cz + b // 9 - 1
            if 0 <= x < ncx and 0 <= y < ncx and 0 <= z < ncx:
                cj = (z * ncx + y) * ncx + x
                D[ci * L:(ci + 1) * L, cj * L:(cj + 1) * L] = Ac[ci, b]
    want = np.array(gold["ac_evals"])
    ed = np.linalg.eigvalsh(0.5 * (D + D.T))
    err = np.abs(ed - want).max() / np.abs(want).max()
    print(f"  A_c spectrum: max rel err {err:.2e}")
    assert err <= 1e-9


@pytest.mark.parametrize("name", list(GOLD))
def test_tpfa_production_preconditioner_matches_oracle(name):
    print(f"case tpfa production precondition {name}", flush=True)
    gold = GOLD[name]
    s, n, rho = _solver(name)
    r = np.random.default_rng(4).standard_normal(n ** 3)
    z = s.precondition(to_dev(r)).cpu().numpy()
    w = np.random.default_rng(5).standard_normal(n ** 3)
    g = gold["precondition"]
    bound = max(1e-10, 100 * gold["subspace_error_bound"])
    e_norm = abs(np.linalg.norm(z) - g["norm"]) / g["norm"]
    e_proj = abs(w @ z - g["w_dot"]) / (np.linalg.norm(w) * g["norm"])
    zs, want = z[np.array(g["idx"])], np.array(g["z"])
    e_samp = np.linalg.norm(zs - want) / np.linalg.norm(want)
    print(f"  |z| {e_norm:.2e}  w^T z {e_proj:.2e}  samples {e_samp:.2e}  bound {bound:.2e}")
    assert e_norm <= bound and e_proj <= bound and e_samp <= bound


@pytest.mark.parametrize("name", list(GOLD))
def test_tpfa_production_iterations_match_oracle(name):
    print(f"case tpfa production iterations {name}", flush=True)
    gold = GOLD[name]
    want = gold["pcg"]["iterations"]
    assert gold["pcg"]["status"] == "converged"
    s, n, rho = _solver(name)
    f = s.heat_source_load(gold["pcg"]["f0"])
    _, info = s.solve(f, rtol=gold["pcg"]["rtol"], maxit=2000)
    print(f"  gpu {info.iterations} (restarts {info.restarts}) oracle {want}")
    assert info.code == 0 and abs(info.iterations - want) <= 1
    assert info.rel_res <= gold["pcg"]["rtol"]
