"""Write tests/golden/tpfa_hierarchy.json: oracle values of the cell-centred
TPFA discretisation at the shipped hierarchy (coarse cells of H = 8 cells,
sd = 8 coarse cells per coarse-coarse cell, L_c = 4, L_cc = 17, smoothing
interval [0.2, 2]) that the GPU parity tests compare with.

Calls only the oracle (oracle/) and the input generators (synth/); nothing here
comes from the HIP path.  Run from the repository root:

    python tests/golden/make_tpfa_golden.py [case ...]

Per case (seeded synthetic field, T_D = 100 on the bottom-patch faces, the
paper's source f0 (1 - rho^3), f0 = 1):
  * n_c, n_cc, the smallest spectral gaps of both levels and the
    subspace-error bound residual / gap;
  * the coarse-coarse eigenvalues and the spectra of A_cc and A_c;
  * one application of Algorithm 1, z = M^-1 r, to r ~ N(0, 1) (seed 4):
    ||z||, w^T z for w ~ N(0, 1) (seed 5) and z at 512 cells (seed 6);
  * PCG iterations to the true relative residual 1e-8 from a zero guess.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import q1, tpfa  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tpfa_hierarchy.json")

CASES = {
    "tpfa_cube64_grf4_c1e6": dict(n=64, kind="grf", ell=4, seed=0, kmin=1e-6),
    "tpfa_cube64_noise_c1e3": dict(n=64, kind="noise", seed=0, kmin=1e-3),
}
KMAX, P, RTOL, TD, F0 = 1.0, 3, 1e-8, 100.0, 1.0
SAMPLES = 512


def field(c):
    n = c["n"]
    if c["kind"] == "noise":
        return synth.uniform_noise_rho(n, c["seed"]).ravel()
    return synth.grf_rho(n, c["ell"], seed=c["seed"]).ravel()


def subspace_error_bound(g, h, tol=1e-12):
    """Eigenvector error ~ residual / gap of both spectral levels (the TPFA
    local problems' Gershgorin bound 2 (1 + sqrt 2) sum_d 1/h_d^2)."""
    b1 = 2 * (1 + np.sqrt(2)) * (1 / g.hx ** 2 + 1 / g.hy ** 2 + 1 / g.hz ** 2)
    e1 = max(tol * b1 / gp for gp in h.cell_gaps)
    e2 = max(tol * nrm / gp for gp, nrm in zip(h.cc_gaps, h.cc_norms))
    return max(e1, e2)


def make(name):
    c = CASES[name]
    n = c["n"]
    rho = field(c)
    flags = synth.dirichlet_patch_faces(n, n, n).ravel()
    g = q1.Grid(n)
    t0 = time.perf_counter()
    h = tpfa.Hierarchy(g, rho, c["kmin"], KMAX, P, flags, tpfa.default_options(H=8, sd=8, Lc=4, Lcc=17))
    t1 = time.perf_counter()
    rec = dict(case=c, n_c=int(h.n_c), n_cc=int(h.n_cc), min_cell_gap=float(min(h.cell_gaps)),
               min_cc_gap=float(min(h.cc_gaps)), subspace_error_bound=subspace_error_bound(g, h))
    rec["cc_evals"] = [float(v) for v in np.concatenate(h.cc_evals)]
    rec["acc_evals"] = [float(v) for v in np.linalg.eigvalsh(h.Acc)]
    rec["ac_evals"] = [float(v) for v in np.linalg.eigvalsh(h.Ac.toarray())]
    r = np.random.default_rng(4).standard_normal(g.nelem)
    z = h.precondition(r)
    w = np.random.default_rng(5).standard_normal(g.nelem)
    idx = np.sort(np.random.default_rng(6).choice(g.nelem, SAMPLES, replace=False))
    rec["precondition"] = dict(norm=float(np.linalg.norm(z)), w_dot=float(w @ z), idx=[int(i) for i in idx],
                               z=[float(v) for v in z[idx]])
    t2 = time.perf_counter()
    f = tpfa.cell_load(g, F0 * (1.0 - rho ** P))
    _, res, _ = tpfa.solve(g, rho, f, flags, c["kmin"], KMAX, P, hier=h, rtol=RTOL, maxit=2000, td=TD)
    t3 = time.perf_counter()
    rec["pcg"] = dict(rtol=RTOL, iterations=int(res.iterations), status=res.status, rel_res=float(res.rel_res),
                      td=TD, f0=F0)
    rec["oracle_seconds"] = dict(setup=t1 - t0, precondition=t2 - t1, solve=t3 - t2)
    print(f"{name}: n_c {h.n_c} n_cc {h.n_cc} iterations {res.iterations} ({res.status}) "
          f"setup {t1 - t0:.1f} s solve {t3 - t2:.1f} s", flush=True)
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    for name in names or list(CASES):
        data[name] = make(name)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=0)
            fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
