"""Benchmark: PCG with the three-grid multiscale preconditioner on the 256^3
Q1 SIMP heat-conduction problem at conductivity contrast 1e6.

One step = set-up for the density field (per-cell spectral problems, coarse
operators) + PCG solve to true relative residual 1e-8 from a zero guess +
compliance sensitivities, on the mixed-precision path (FP64 outer PCG with a
double-double iterate, FP32 cycle, BF16 density and basis copies, FP64
coarse-coarse solve).  value = free DOFs / solve time (set-up excluded, as the
metric defines it).  The all-FP64 path is timed on the same field for
comparison.  The CPU oracle is timed on a bounded sample (rank 0, N = 1).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

N = 256
ELL = 16
KMIN = 1e-6
RTOL = 1e-8
HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline():
    """Oracle PCG-MsMG solve of a bounded sample; DOFs/s of the solve.

    The oracle runs as it stands (NumPy/SciPy, FP64 with an extended-precision
    iterate) with BLAS limited to one thread, so `cores` is 1."""
    import threadpoolctl

    from oracle import msmg as omsmg
    from oracle import q1

    n = 64
    ell = ELL * n / N  # same feature size relative to the box as the 256^3 field
    g = q1.Grid(n)
    rho = synth.grf_rho(n, ell, seed=0).ravel()
    mask = synth.dirichlet_patch_mask(n, n, n).ravel()
    f = q1.element_load(g, 1.0)
    with threadpoolctl.threadpool_limits(limits=1):
        t0 = time.perf_counter()
        h = omsmg.Hierarchy(g, rho, KMIN, 1.0, 3, mask, omsmg.Options(H=8, sd=8))
        t1 = time.perf_counter()
        T, res, _ = omsmg.solve(g, rho, f, mask, KMIN, 1.0, 3, hier=h, rtol=RTOL, maxit=1000)
        t2 = time.perf_counter()
    free = int(g.nnodes - mask.sum())
    return {
        "value": free / (t2 - t1),
        "unit": "DOFs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle PCG-MsMG solve (FP64, extended-precision iterate) of a {n}^3 thresholded GRF "
                   f"(ell={ell:g} elements, contrast 1e6, H=8, sd=8), rtol {RTOL}, {res.iterations} iterations, "
                   f"status {res.status}, one thread; set-up {t1 - t0:.1f} s excluded"),
        "solve_s": t2 - t1,
        "setup_s": t1 - t0,
    }


SOURCES_FOR_TRAFFIC = ("paper_2410_06850_amd/csrc/fine_kernels.hip", "paper_2410_06850_amd/csrc/march.h",
                       "paper_2410_06850_amd/csrc/common.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_apply_cube256_grf16_c1e6_traffic.json")


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for rel in SOURCES_FOR_TRAFFIC:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per operator-apply launch from the committed rocprofv3 counter
    runs (FETCH_SIZE, WRITE_SIZE scaled by a plain-copy calibration), or None
    when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


PATHS = {
    # FP64 cycle arithmetic with BF16 copies of k and R_c, FP32 Jacobi diagonal
    "mixed": dict(vcycle_dtype=0, rho_v_dtype=2, basis_dtype=2),
    "fp64": dict(),
    # FP32 cycle vectors and arithmetic (BF16 copies)
    "f32cycle": dict(vcycle_dtype=1, rho_v_dtype=2, basis_dtype=2),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison path")
    ap.add_argument("--no-f32", action="store_true", help="skip the FP32-cycle comparison path")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (sharding is described in the design "
              "notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2410_06850_amd as pkg

    n = args.n
    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    _log(f"generating the {n}^3 field")
    rho_np = synth.grf_rho(n, ELL * n / N, seed=0).ravel()
    mask_np = synth.dirichlet_patch_mask(n, n, n).ravel()
    free = int((n + 1) ** 3 - int(mask_np.sum()))
    rho = torch.tensor(rho_np, device=dev)
    mask = torch.tensor(mask_np, device=dev)

    def run_path(opts, steps, warmup, tag):
        s = pkg.Solver(n, timing=1, tune_cache=os.path.join(ROOT, "gpurun_out", "tune_cache.txt"), **opts)
        f = s.element_load(const=1.0)
        T = torch.empty_like(f)
        recs = []
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.setup(rho, KMIN, 1.0, 3, mask)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            T, info = s.solve(f, T, rtol=RTOL, maxit=1000)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            dc = s.sensitivity(T)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            _log(f"{tag} step {k}: setup {1e3 * (t1 - t0):.1f} ms, solve {1e3 * (t2 - t1):.1f} ms "
                 f"({info.iterations} it, rel.res {info.rel_res:.2e}, code {info.code}), "
                 f"sensitivity {1e3 * (t3 - t2):.1f} ms, apply {info.apply_ms * 1e3:.1f} us")
            if info.code != 0:
                raise RuntimeError(f"{tag}: solve did not converge: {dict(info)}")
            if k >= warmup:
                recs.append(dict(setup=t1 - t0, solve=t2 - t1, sens=t3 - t2, step=t3 - t0, info=dict(info)))
        del dc, s
        torch.cuda.empty_cache()
        return recs

    def summary(recs):
        last = recs[-1]["info"]
        t = float(np.mean([r["solve"] for r in recs]))
        return {
            "value": free / t,
            "iterations": last["iterations"],
            "rel_res": last["rel_res"],
            "solve_ms": 1e3 * t,
            "setup_ms": 1e3 * float(np.mean([r["setup"] for r in recs])),
            "sensitivity_ms": 1e3 * float(np.mean([r["sens"] for r in recs])),
            "apply_us": 1e3 * float(np.mean([r["info"]["apply_ms"] for r in recs])),
            "precond_us": 1e3 * float(np.mean([r["info"]["precond_ms"] for r in recs])),
        }

    _log("mixed-precision path")
    mix = run_path(PATHS["mixed"], args.steps, args.warmup, "mixed")
    t_solve = float(np.mean([r["solve"] for r in mix]))
    t_step = float(np.mean([r["step"] for r in mix]))
    info = mix[-1]["info"]
    # dominant kernel: the PCG operator apply (one launch per iteration), timed
    # with HIP events on the solve stream inside the timed steps
    apply_ms = float(np.mean([r["info"]["apply_ms"] for r in mix]))
    nn, ne = (n + 1) ** 3, n ** 3
    apply_bytes = 16 * nn + 8 * ne + nn / 8  # x read, y write, k read, mask bits
    achieved = apply_bytes / (apply_ms * 1e-3) / 1e9
    traffic = measured_traffic() if n == N else None

    others = {}
    if not args.no_fp64:
        _log("FP64 path")
        others["fp64"] = summary(run_path(PATHS["fp64"], 1, 0, "fp64"))
    if not args.no_f32:
        _log("FP32-cycle path")
        others["f32cycle"] = summary(run_path(PATHS["f32cycle"], 1, 0, "f32cycle"))

    cpu = None
    if not args.no_cpu_baseline:
        _log("CPU oracle baseline")
        cpu = cpu_baseline()

    out = {
        "metric": "DOFs/s solved to rel-res 1e-8 at 256^3, contrast 1e6: FP64 vs mixed V-cycle",
        "value": free / t_solve,
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"cube{n}_grf{ELL * n // N}_c1e6",
            "elements": n ** 3,
            "free_dofs": free,
            "field": f"thresholded Gaussian random field, ell={ELL * n / N:g} elements, volume fraction 0.4, seed 0",
            "k_min": KMIN, "k_max": 1.0, "p": 3, "rtol": RTOL,
            "hierarchy": {"H": 8, "sd": 8, "Lc": 4, "Lcc": 17, "cheb_degree": 2},
            "precision": ("FP64 PCG (double-double iterate) and FP64 cycle arithmetic; BF16 copies of k and R_c, "
                          "FP32 Jacobi diagonal in the cycle; FP64 coarse levels"),
            "step": "set-up + PCG solve from zero + compliance sensitivity; value counts the solve only",
        },
        "iterations": info["iterations"],
        "rel_res": info["rel_res"],
        "solve_ms": 1e3 * t_solve,
        "setup_ms": 1e3 * float(np.mean([r["setup"] for r in mix])),
        "precond_us": 1e3 * float(np.mean([r["info"]["precond_ms"] for r in mix])),
        "paths": others,
        "roofline": {
            "kernel": "k_apply (PCG operator apply, FP64, difference form)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "apply_us": apply_ms * 1e3,
            "bytes_per_launch": apply_bytes,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
