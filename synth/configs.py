"""Workload configurations of the model problem (sizes, contrasts, generators).

Each entry names the mesh, the density generator and its parameters, the
material bounds, the stopping tolerance and the hierarchy sizes.  Material law
k = k_min + rho^p (k_max - k_min) with p = 3, k_max = 1; source f = 1; zero
temperature on the 0.2 x 0.2 bottom patch.
"""
from __future__ import annotations

WORKLOADS = {
    "cube16_noise": dict(
        n=16, gen="noise", seeds=(0, 1, 2), kmin=1e-3, kmax=1.0, p=3,
        rtol=1e-10, precision="fp64", H=8, sd=2, Lc=4, Lcc=17,
    ),
    "cube128_grf8_c1e6": dict(
        n=128, gen="grf", ell=8, seeds=(0, 1, 2), kmin=1e-6, kmax=1.0, p=3,
        rtol=1e-8, precision="fp64", H=8, sd=8, Lc=4, Lcc=17,
    ),
    "cube256_grf16": dict(
        n=256, gen="grf", ell=16, seeds=(0, 1, 2), kmins=(1e-2, 1e-4, 1e-6),
        kmin=1e-6, kmax=1.0, p=3, rtol=1e-8, precision="mixed", H=8, sd=8,
        Lc=4, Lcc=17,
    ),
    "cube512_to": dict(
        n=512, gen="const", base=0.3, kmin=1e-6, kmax=1.0, p=3, rtol=1e-8,
        precision="mixed", H=8, sd=8, Lc=4, Lcc=17, to_iters=20,
        filter_radius=1.5, volfrac=0.3,
    ),
    "cube1024_grf32_c1e6": dict(
        n=1024, gen="grf", ell=32, seeds=(0,), kmin=1e-6, kmax=1.0, p=3,
        rtol=1e-8, precision="mixed", H=8, sd=16, Lc=4, Lcc=17,
    ),
}


def workload(name):
    return dict(WORKLOADS[name])
