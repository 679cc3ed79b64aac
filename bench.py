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
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

# launch-shape cache of the level-1 eigensolver tuner (a host file; the first
# set-up of a handle without a cached entry times the candidates)
TUNE_CACHE = os.environ.get("MSMG_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "msmg_tune_cache.txt"))

N = 256
ELL = 16
KMIN = 1e-6
RTOL = 1e-8
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # dense FP64 (matrix cores)


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The oracle (NumPy/SciPy, FP64 with an extended-precision iterate, as it
    stands) timed on the host: set-up and PCG-MsMG solve of the 16^3 noise case
    (k_min 1e-3, H 8, sd 2, rtol 1e-10) and of a 64^3 thresholded GRF at
    contrast 1e6 (ell 4, the benchmark field's feature size relative to the
    box, H 8, sd 8, rtol 1e-8), each with BLAS on one thread and on every host
    core.  `value` = DOFs/s of the 64^3 solve on every core; the 128^3 and
    256^3 oracle solves take many minutes and are left out of the bench run."""
    import threadpoolctl

    from oracle import msmg as omsmg
    from oracle import q1

    nproc = os.cpu_count() or 1
    runs = []
    for n, kind, kmin, H, sd, rtol in ((16, "noise", 1e-3, 8, 2, 1e-10), (64, "grf", KMIN, 8, 8, RTOL)):
        g = q1.Grid(n)
        rho = (synth.uniform_noise_rho(n, 0) if kind == "noise" else synth.grf_rho(n, ELL * n / N, seed=0)).ravel()
        mask = synth.dirichlet_patch_mask(n, n, n).ravel()
        f = q1.element_load(g, 1.0)
        free = int(g.nnodes - mask.sum())
        for threads in (1, nproc):
            with threadpoolctl.threadpool_limits(limits=threads):
                t0 = time.perf_counter()
                h = omsmg.Hierarchy(g, rho, kmin, 1.0, 3, mask, omsmg.Options(H=H, sd=sd))
                t1 = time.perf_counter()
                _, res, _ = omsmg.solve(g, rho, f, mask, kmin, 1.0, 3, hier=h, rtol=rtol, maxit=1000)
                t2 = time.perf_counter()
            runs.append(dict(n=n, field=kind, k_min=kmin, H=H, sd=sd, rtol=rtol, threads=threads,
                             iterations=res.iterations, status=res.status, setup_s=t1 - t0, solve_s=t2 - t1,
                             dofs_per_s=free / (t2 - t1)))
            _log(f"oracle {n}^3 {kind}, {threads} thread(s): set-up {t1 - t0:.1f} s, solve {t2 - t1:.1f} s, "
                 f"{res.iterations} iterations")
    head = runs[-1]
    return {
        "value": head["dofs_per_s"],
        "unit": "DOFs/s",
        "cores": nproc,
        "kind": "oracle",
        "sample": (f"oracle PCG-MsMG solve (FP64, extended-precision iterate) of a 64^3 thresholded GRF "
                   f"(ell={ELL * 64 / N:g} elements, contrast 1e6, H=8, sd=8), rtol {RTOL}, {head['iterations']} "
                   f"iterations, BLAS on {nproc} threads (sparse products single-threaded); set-up excluded"),
        "nproc": nproc,
        "cpu_model": _cpu_model(),
        "runs": runs,
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
    # FP64 cycle arithmetic with a BF16 copy of k, an FP32 copy of R_c and an
    # FP32 Jacobi diagonal
    "mixed": dict(vcycle_dtype=0, rho_v_dtype=2, basis_dtype=1),
    "fp64": dict(),
    # the same with a BF16 basis as well: less traffic, but the rounded coarse
    # basis costs iterations on fields with large high-conductivity regions
    "bf16": dict(vcycle_dtype=0, rho_v_dtype=2, basis_dtype=2),
    # FP32 copies of both
    "f32": dict(vcycle_dtype=0, rho_v_dtype=1, basis_dtype=1),
    # FP32 cycle vectors and arithmetic (BF16 copies)
    "f32cycle": dict(vcycle_dtype=1, rho_v_dtype=2, basis_dtype=2),
}


def run_workload(name, args):
    """Companion workloads (one JSON line each): the 128^3 FP64 runs, the 256^3
    contrast sweep, the 512^3 optimisation loop."""
    import torch

    import paper_2410_06850_amd as pkg

    dev = torch.device("cuda", 0)
    tune = TUNE_CACHE
    out = {"workload": name, "runs": []}

    def solve_case(n, rho_np, kmin, opts, rtol=RTOL, seed=None, tag=""):
        mask_np = synth.dirichlet_patch_mask(n, n, n).ravel()
        free = int((n + 1) ** 3 - int(mask_np.sum()))
        s = pkg.Solver(n, tune_cache=tune, **opts)
        rho = torch.tensor(rho_np, device=dev)
        mask = torch.tensor(mask_np, device=dev)
        f = s.element_load(const=1.0)
        rec = {}
        for rep in range(2):  # the second repetition is reported (first one tunes and warms up)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.setup(rho, kmin, 1.0, 3, mask)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            T, info = s.solve(f, rtol=rtol, maxit=2000)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec = dict(tag=tag, n=n, seed=seed, k_min=kmin, iterations=info.iterations, code=info.code,
                       rel_res=info.rel_res, setup_ms=1e3 * (t1 - t0), solve_ms=1e3 * (t2 - t1),
                       dofs_per_s=free / (t2 - t1))
        _log(json.dumps(rec))
        del s
        torch.cuda.empty_cache()
        return rec

    mixed, fp64, bf16 = PATHS["mixed"], PATHS["fp64"], PATHS["bf16"]
    # coefficient copies of the single-path workloads (interpolation,
    # optimisation, continuation, 1024^3): BF16 k and R_c unless --copies
    # f32 (FP32 both) or mixed (BF16 k, FP32 R_c)
    lean = {"bf16": bf16, "f32": PATHS["f32"], "mixed": mixed}[args.copies]
    if name == "cube128_grf8_c1e6":
        for seed in (0, 1, 2):
            rho = synth.grf_rho(128, 8, seed=seed).ravel()
            out["runs"].append(solve_case(128, rho, 1e-6, fp64, seed=seed, tag="fp64"))
            out["runs"].append(solve_case(128, rho, 1e-6, mixed, seed=seed, tag="mixed"))
            out["runs"].append(solve_case(128, rho, 1e-6, bf16, seed=seed, tag="bf16"))
    elif name == "cube256_grf16_contrast_sweep":
        rho = synth.grf_rho(256, 16, seed=0).ravel()
        for kmin in (1e-2, 1e-4, 1e-6):
            out["runs"].append(solve_case(256, rho, kmin, fp64, tag="fp64"))
            out["runs"].append(solve_case(256, rho, kmin, mixed, tag="mixed"))
            out["runs"].append(solve_case(256, rho, kmin, bf16, tag="bf16"))
    elif name == "cube256_grf16_paper_pair":
        # the paper's own state and adjoint pair: source f0 (1 - rho^p) with
        # f0 = 1, T_D = 100 on the patch (LS1), mean-temperature adjoint (LS2)
        # sharing the set-up, then the sensitivity with its df/drho term
        n = 256
        rho_np = synth.grf_rho(n, 16, seed=0).ravel()
        mask_np = synth.dirichlet_patch_mask(n, n, n).ravel()
        free = int((n + 1) ** 3 - int(mask_np.sum()))
        rho = torch.tensor(rho_np, device=dev)
        mask = torch.tensor(mask_np, device=dev)
        td = torch.where(mask != 0, 100.0, 0.0).to(torch.float64)
        for kmin in (1e-2, 1e-4, 1e-6):
            for tag, opts in (("fp64", fp64), ("mixed", mixed), ("bf16", bf16)):
                # pair_rhs: the handle also carries the second vector set of
                # the batched pair, timed after the two sequential solves
                s = pkg.Solver(n, tune_cache=tune, pair_rhs=1, **opts)
                rec = {}
                for rep in range(2):  # the second repetition is reported
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s.setup(rho, kmin, 1.0, 3, mask, td)
                    f = s.heat_source_load(1.0)
                    w = s.mean_temperature_weights()
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    T, i1 = s.solve(f, rtol=RTOL, maxit=2000)
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                    u, i2 = s.solve_adjoint(w, rtol=RTOL, maxit=2000)
                    torch.cuda.synchronize()
                    t3 = time.perf_counter()
                    dc = s.sensitivity_heat_source(T, u, 1.0)
                    torch.cuda.synchronize()
                    t4 = time.perf_counter()
                    Tp, up, j1, j2 = s.solve_pair(f, w, rtol=RTOL, maxit=2000)
                    torch.cuda.synchronize()
                    t5 = time.perf_counter()
                    rec = dict(tag=tag, n=n, k_min=kmin, mean_T=float(torch.dot(w, T)),
                               setup_ms=1e3 * (t1 - t0), ls1_iterations=i1.iterations, ls1_ms=1e3 * (t2 - t1),
                               ls1_rel_res=i1.rel_res, ls2_iterations=i2.iterations, ls2_ms=1e3 * (t3 - t2),
                               ls2_rel_res=i2.rel_res, sensitivity_ms=1e3 * (t4 - t3),
                               codes=[i1.code, i2.code], dofs_per_s=2 * free / (t3 - t1),
                               dc_min=float(dc.min()), dc_max=float(dc.max()),
                               pair_ms=1e3 * (t5 - t4), pair_iterations=[j1.iterations, j2.iterations],
                               pair_codes=[j1.code, j2.code], pair_dofs_per_s=2 * free / (t5 - t4),
                               pair_speedup=(t3 - t1) / (t5 - t4),
                               pair_bitwise_equal=bool(torch.equal(T, Tp) and torch.equal(u, up)))
                _log(json.dumps(rec))
                out["runs"].append(rec)
                del s, T, u, dc, Tp, up
                torch.cuda.empty_cache()
    elif name == "cube512_paper_contrasts":
        # the paper's solver-comparison setting at its size and tolerance:
        # 512^3, contrast 10^cr for cr = 1..6, source f0 (1 - rho^p), T_D = 100,
        # LS1 (state) and LS2 (mean-temperature adjoint) to rtol 1e-6 with one
        # set-up; the paper's fields come from its optimisation runs and are
        # replaced by a thresholded GRF (ell 32, volume fraction 0.4)
        n = 512
        rho = torch.tensor(synth.grf_rho(n, 32, seed=0).ravel(), device=dev)
        mask = torch.tensor(synth.dirichlet_patch_mask(n, n, n).ravel(), device=dev)
        free = int((n + 1) ** 3 - int(mask.sum()))
        td = torch.where(mask != 0, 100.0, 0.0).to(torch.float64)
        for tag, opts in (("mixed", mixed), ("bf16", bf16), ("fp64", fp64)):
            s = pkg.Solver(n, tune_cache=tune, **opts)
            s.setup(rho, 1e-1, 1.0, 3, mask, td)  # launch-shape tuning, not timed
            for cr in range(1, 7):
                kmin = 10.0 ** (-cr)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.setup(rho, kmin, 1.0, 3, mask, td)
                f = s.heat_source_load(1.0)
                w = s.mean_temperature_weights()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                T, i1 = s.solve(f, rtol=1e-6, maxit=4000)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                u, i2 = s.solve_adjoint(w, rtol=1e-6, maxit=4000)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                rec = dict(tag=tag, n=n, cr=cr, setup_s=t1 - t0, ls1_s=t2 - t1, ls1_iterations=i1.iterations,
                           ls2_s=t3 - t2, ls2_iterations=i2.iterations, codes=[i1.code, i2.code],
                           ls1_rel_res=i1.rel_res, ls2_rel_res=i2.rel_res, free_dofs=free)
                _log(json.dumps(rec))
                out["runs"].append(rec)
                del T, u
            s.close()
            del s
            torch.cuda.empty_cache()
    elif name == "cube512_tpfa_paper_contrasts":
        # the same setting on the paper's own discretisation (cell-centred
        # TPFA, FP64): 512^3 cells, contrast 10^cr for cr = 1..6, T_D = 100 on
        # the bottom-patch faces, source f0 (1 - rho^p), LS1 and LS2 to rtol
        # 1e-6 with one set-up, hierarchies (sd, L_c, L_cc) = (8, 4, 17) and
        # (6, 4, 17) with H = 8 (the paper's best columns)
        n = 512
        rho = torch.tensor(synth.grf_rho(n, 32, seed=0).ravel(), device=dev)
        flags = torch.tensor(synth.dirichlet_patch_faces(n, n, n).ravel(), device=dev)
        td = torch.full((n ** 3,), 100.0, dtype=torch.float64, device=dev)
        for sd in (8, 6):
            s = pkg.Solver(n, discretisation="tpfa", sd=sd, tune_cache=tune)
            s.setup(rho, 1e-1, 1.0, 3, flags, td)  # launch-shape tuning, not timed
            for cr in range(1, 7):
                kmin = 10.0 ** (-cr)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.setup(rho, kmin, 1.0, 3, flags, td)
                f = s.heat_source_load(1.0)
                w = s.mean_temperature_weights()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                T, i1 = s.solve(f, rtol=1e-6, maxit=4000)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                u, i2 = s.solve_adjoint(w, rtol=1e-6, maxit=4000)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
                rec = dict(tag=f"tpfa_sd{sd}", n=n, cr=cr, sd=sd, Lc=4, Lcc=17, setup_s=t1 - t0, ls1_s=t2 - t1,
                           ls1_iterations=i1.iterations, ls2_s=t3 - t2, ls2_iterations=i2.iterations,
                           codes=[i1.code, i2.code], ls1_rel_res=i1.rel_res, ls2_rel_res=i2.rel_res, cells=n ** 3)
                _log(json.dumps(rec))
                out["runs"].append(rec)
                del T, u
            s.close()
            del s
            torch.cuda.empty_cache()
    elif name == "cube256_adaptive_basis":
        # the adaptive local basis size (options.lc_threshold) against fixed
        # L_c on the benchmark's field, Q1 (mixed path) and TPFA (FP64,
        # T_D = 0, source f0 (1 - rho^3)): effective coarse dimension,
        # iterations to 1e-8, set-up and solve time
        n = 256
        rho = torch.tensor(synth.grf_rho(n, 16, seed=0).ravel(), device=dev)
        for disc in ("q1", "tpfa"):
            if disc == "q1":
                mask = torch.tensor(synth.dirichlet_patch_mask(n, n, n).ravel(), device=dev)
                base = dict(mixed)
            else:
                mask = torch.tensor(synth.dirichlet_patch_faces(n, n, n).ravel(), device=dev)
                base = dict(discretisation="tpfa")
            for cfg in (dict(Lc=4), dict(Lc=7, lc_threshold=0.5), dict(Lc=7, lc_threshold=1.0),
                        dict(Lc=7, lc_threshold=2.0), dict(Lc=7)):
                s = pkg.Solver(n, tune_cache=tune, **base, **cfg)
                s.setup(rho, KMIN, 1.0, 3, mask)  # launch-shape tuning, not timed
                f = s.element_load(const=1.0) if disc == "q1" else s.heat_source_load(1.0)
                for rep in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s.setup(rho, KMIN, 1.0, 3, mask)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    T, info = s.solve(f, rtol=RTOL, maxit=2000)
                    torch.cuda.synchronize()
                    t2 = time.perf_counter()
                st = s.export(5, s.plan().ncells, torch.int32).numpy()
                cnt = (st >> 20) & 0xFF
                rec = dict(disc=disc, cfg=cfg, n_c_effective=int(cnt.sum()), basis_sizes=np.bincount(cnt).tolist(),
                           setup_ms=1e3 * (t1 - t0), solve_ms=1e3 * (t2 - t1), iterations=info.iterations,
                           rel_res=info.rel_res, code=info.code)
                _log(json.dumps(rec))
                out["runs"].append(rec)
                s.close()
                del s, T
                torch.cuda.empty_cache()
    elif name == "cube512_topopt":
        n = 512
        s = pkg.Solver(n, tune_cache=tune, eig_warm_start=1, **lean)
        mask = torch.tensor(synth.dirichlet_patch_mask(n, n, n).ravel(), device=dev)
        t0 = time.perf_counter()
        _, hist = pkg.topopt.optimize(s, mask, iterations=args.iterations, volume_fraction=0.3, x0=0.3,
                                      radius=1.5, kmin=1e-6, optimizer=args.optimizer,
                                      log=lambda r: _log(json.dumps(r)))
        out["total_s"] = time.perf_counter() - t0
        out["runs"] = hist
        out["config"] = dict(n=n, iterations=args.iterations, volume_fraction=0.3, radius=1.5, move=0.2, eta=0.5,
                             k_min=1e-6, precision=f"mixed, {args.copies} copies", eig_warm_start=1,
                             update=args.optimizer.upper())
    elif name in ("cube128_to_512_continuation", "cube128_to_512_tpfa_continuation"):
        # the interpolation technique at the design level (section 4): the
        # paper's mean-temperature problem (source f0 (1 - rho^p), T_D = 100,
        # contrast 1e6, volume fraction 0.05) optimised 40 / 20 / 10 iterations
        # on 128^3 / 256^3 / 512^3, each level started from the injected
        # design of the previous one; then 10 iterations directly on 512^3
        # from the uniform design for comparison (design update: --optimizer,
        # the paper's MMA by default); the _tpfa_ variant on the paper's
        # cell-centred discretisation (FP64)
        vf = 0.05
        use_tpfa = "tpfa" in name

        def make_mask(n):
            if use_tpfa:
                return torch.tensor(synth.dirichlet_patch_faces(n, n, n).ravel(), device=dev)
            return torch.tensor(synth.dirichlet_patch_mask(n, n, n).ravel(), device=dev)

        def make_solver(n):
            if use_tpfa:
                return pkg.Solver(n, discretisation="tpfa", tune_cache=tune, eig_warm_start=1)
            return pkg.Solver(n, tune_cache=tune, eig_warm_start=1, **lean)

        def make_fixed(n):
            if use_tpfa:
                return torch.full((n ** 3,), 100.0, dtype=torch.float64, device=dev)
            return torch.where(make_mask(n) != 0, 100.0, 0.0).to(torch.float64)

        def summary(lv):
            h = lv["history"]
            return dict(n=lv["n"], iterations=lv["iterations"], seconds=lv["seconds"], first=h[0]["objective"],
                        last=h[-1]["objective"], volume=h[-1]["volume"], pcg=[r["pcg_iterations"] for r in h],
                        adjoint=[r["adjoint_iterations"] for r in h])

        common = dict(kmin=1e-6, objective="mean_temperature", f0=1.0, maxit=4000, optimizer=args.optimizer,
                      log=lambda r: _log(json.dumps(r)))
        t_all = time.perf_counter()
        x, levels = pkg.topopt.continuation(make_solver, make_mask, 128, (40, 20, 10), vf, make_fixed=make_fixed,
                                            **common)
        total_cont = time.perf_counter() - t_all
        del x
        torch.cuda.empty_cache()
        _, direct = pkg.topopt.continuation(make_solver, make_mask, 512, (10,), vf, make_fixed=make_fixed, **common)
        levels = [summary(lv) for lv in levels]
        direct = summary(direct[0])
        out["runs"] = [dict(kind="continuation", total_s=total_cont, levels=levels),
                       dict(kind="direct512", **direct)]
        out["config"] = dict(schedule=[40, 20, 10], volume_fraction=vf, k_min=1e-6, T_D=100.0, f0=1.0, radius=1.5,
                             move=0.2, eta=0.5, update=args.optimizer.upper(),
                             discretisation="TPFA" if use_tpfa else "Q1",
                             precision="FP64" if use_tpfa else f"mixed, {args.copies} copies")
    elif name == "cube512_grf32_warmstart":
        # the interpolation step: solve the 256^3 companion (2^3 block average of
        # the same unthresholded field, thresholded at its own 60th percentile),
        # prolong T to 512^3 (trilinear) and start the 512^3 solve from it
        w = synth.grf_raw(512, 32, seed=0)
        rho_f = synth.threshold_field(w).ravel()
        rho_c = synth.threshold_field(synth.block_average(w)).ravel()
        del w
        res = {}
        for n, rho_np in ((256, rho_c), (512, rho_f)):
            mask_np = synth.dirichlet_patch_mask(n, n, n).ravel()
            s = pkg.Solver(n, tune_cache=tune, **lean)
            s.setup(torch.tensor(rho_np, device=dev), 1e-6, 1.0, 3, torch.tensor(mask_np, device=dev))
            f = s.element_load(const=1.0)
            if n == 256:
                T, info = s.solve(f, rtol=RTOL, maxit=2000)
                res["coarse"] = dict(n=n, iterations=info.iterations, solve_ms=info.solve_ms)
                x0 = pkg.prolong_nodal(T, (n, n, n))
                del T
            else:
                T, cold = s.solve(f, rtol=RTOL, maxit=2000)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                T, warm = s.solve(f, x0, rtol=RTOL, maxit=2000, use_x0=True)
                torch.cuda.synchronize()
                tw = time.perf_counter() - t0
                res["fine_cold"] = dict(n=n, iterations=cold.iterations, solve_ms=cold.solve_ms, code=cold.code,
                                        rel_res=cold.rel_res)
                res["fine_warm"] = dict(n=n, iterations=warm.iterations, solve_ms=1e3 * tw, code=warm.code,
                                        rel_res=warm.rel_res)
                res["setup_ms"] = cold.setup_ms
            _log(json.dumps(res))
            del s
            torch.cuda.empty_cache()
        out["runs"] = [res]
    elif name == "cube1024_grf32_c1e6":
        # the largest one-GPU instance: 1024^3 elements, FP32 canonical density
        # (GRF ell 32, contrast 1e6), lean memory layout; the 512^3 companion
        # (2^3 block average of the same unthresholded field, thresholded at its
        # own 60th percentile) is solved first and its T prolonged (trilinear)
        # as the warm start; a cold start is run as well
        t0 = time.perf_counter()
        w = synth.grf_raw(1024, 32, seed=0, dtype=np.float32)
        rho_f = synth.threshold_field(w, dtype=np.float32).ravel()
        rho_c = synth.threshold_field(synth.block_average(w), dtype=np.float32).ravel()
        del w
        _log(json.dumps(dict(stage="fields", s=time.perf_counter() - t0)))
        res = {}
        n = 512
        mask_np = synth.dirichlet_patch_mask(n, n, n).ravel()
        s = pkg.Solver(n, tune_cache=tune, **lean)
        s.setup(torch.tensor(rho_c, device=dev), 1e-6, 1.0, 3, torch.tensor(mask_np, device=dev))
        f = s.element_load(const=1.0)
        T, info = s.solve(f, rtol=RTOL, maxit=2000)
        res["coarse"] = dict(n=n, iterations=info.iterations, solve_ms=info.solve_ms, setup_ms=info.setup_ms,
                             code=info.code)
        _log(json.dumps(res["coarse"]))
        x0 = pkg.prolong_nodal(T, (n, n, n))
        del T, f, s, rho_c
        torch.cuda.empty_cache()
        n = 1024
        opts = dict(lean, rho_storage=1, lean_memory=1, timing=1)
        mask_np = synth.dirichlet_patch_mask(n, n, n).ravel()
        free = int((n + 1) ** 3 - int(mask_np.sum()))
        s = pkg.Solver(n, tune_cache=tune, **opts)
        plan = s.plan()
        rho = torch.from_numpy(rho_f).to(dev)
        mask = torch.from_numpy(mask_np).to(dev)
        del rho_f
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.setup(rho, 1e-6, 1.0, 3, mask)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        _log(json.dumps(dict(stage="setup 1024", s=setup_s, handle_bytes=plan.device_bytes)))
        f = s.element_load(const=1.0)
        T, cold = s.solve(f, rtol=RTOL, maxit=2000)
        res["fine_cold"] = dict(n=n, iterations=cold.iterations, solve_ms=cold.solve_ms, code=cold.code,
                                rel_res=cold.rel_res, dofs_per_s=free / (1e-3 * cold.solve_ms),
                                apply_us=1e3 * cold.apply_ms, precond_us=1e3 * cold.precond_ms,
                                setup_phase_ms=cold.setup_phase_ms)
        _log(json.dumps(res["fine_cold"]))
        T, warm = s.solve(f, x0, rtol=RTOL, maxit=2000, use_x0=True)
        res["fine_warm"] = dict(n=n, iterations=warm.iterations, solve_ms=warm.solve_ms, code=warm.code,
                                rel_res=warm.rel_res, dofs_per_s=free / (1e-3 * warm.solve_ms))
        _log(json.dumps(res["fine_warm"]))
        free_b, total_b = torch.cuda.mem_get_info()
        res["memory"] = dict(handle_bytes=plan.device_bytes, device_used_bytes=total_b - free_b,
                             torch_peak_bytes=torch.cuda.max_memory_allocated(), n_cc=plan.n_cc)
        res["setup_ms"] = 1e3 * setup_s
        res["free_dofs"] = free
        res["eig_unconverged"], res["cc_unconverged"] = warm.eig_unconverged, warm.cc_unconverged
        out["runs"] = [res]
        out["config"] = dict(n=n, ell=32, k_min=1e-6, precision=f"mixed, {args.copies} copies", rho_storage="f32", lean_memory=1,
                             H=8, sd=8, Lc=4, Lcc=17)
    else:
        raise SystemExit(f"unknown workload {name}")
    print(json.dumps(out), flush=True)


def run_tpfa(pkg, rho, n, steps, warmup, rtol=RTOL):
    """The paper's own discretisation, cell-centred TPFA, on the same design
    field: the bottom patch as Dirichlet faces at T_D = 100 and the
    design-dependent heat source f0 (1 - rho^p), f0 = 1 (the state problem of
    the paper's section 4); FP64 throughout.  One step = set-up + solve from
    zero; value counts the solve."""
    import torch

    dev = rho.device
    flags = torch.tensor(synth.dirichlet_patch_faces(n, n, n).ravel(), device=dev)
    td = torch.full((n ** 3,), 100.0, dtype=torch.float64, device=dev)
    s = pkg.Solver(n, discretisation="tpfa", timing=1, tune_cache=TUNE_CACHE)
    T = T_lo = None
    recs = []
    for k in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.setup(rho, KMIN, 1.0, 3, flags, td)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        f = s.heat_source_load(1.0)
        if T is None:
            T, T_lo = torch.empty_like(f), torch.empty_like(f)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        T, info = s.solve(f, T, rtol=rtol, maxit=2000, T_lo=T_lo)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        _log(f"tpfa step {k}: setup {1e3 * (t1 - t0):.1f} ms, solve {1e3 * (t3 - t2):.1f} ms "
             f"({info.iterations} it, rel.res {info.rel_res:.2e}, code {info.code}), apply {info.apply_ms * 1e3:.1f} us")
        if info.code != 0:
            raise RuntimeError(f"tpfa: solve did not converge: {dict(info)}")
        if k >= warmup:
            recs.append(dict(setup=t1 - t0, solve=t3 - t2, info=dict(info)))
    apply_ms = s.time_apply(T, 50)
    _, i6 = s.solve(f, rtol=1e-6, maxit=2000)
    t = float(np.mean([r["solve"] for r in recs]))
    apply_in_solve_ms = float(np.mean([r["info"]["apply_ms"] for r in recs]))
    apply_bytes = 25.0 * n ** 3  # x and k read (8 B each), the face flags (1 B), y written (8 B)
    ach = apply_bytes / (apply_ms * 1e-3) / 1e9
    ph = np.mean([r["info"]["setup_phase_ms"] for r in recs], axis=0)
    del s
    torch.cuda.empty_cache()
    return {
        "workload": f"cube{n}_tpfa_grf{ELL * n // N}_c1e6",
        "discretisation": "cell-centred two-point flux finite volumes (harmonic face conductivities), FP64",
        "problem": "T_D = 100 on the bottom-patch faces, heat source f0 (1 - rho^3), f0 = 1",
        "cells": n ** 3,
        "value": n ** 3 / t,
        "unit": "DOFs/s",
        "iterations": recs[-1]["info"]["iterations"],
        "rel_res": recs[-1]["info"]["rel_res"],
        "iterations_rtol_1e-6": i6.iterations,
        "solve_ms": 1e3 * t,
        "setup_ms": 1e3 * float(np.mean([r["setup"] for r in recs])),
        "setup_phases_ms": {"local_spectral_problems": float(ph[0]), "galerkin_Ac": float(ph[1]),
                            "coarse_coarse_problems": float(ph[2]), "Acc_and_inverse": float(ph[3])},
        "precond_us": 1e3 * float(np.mean([r["info"]["precond_ms"] for r in recs])),
        "roofline": {"kernel": "k_tpfa_apply (PCG operator apply q = A p, FP64, difference form)", "bound": "hbm",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "apply_us": apply_ms * 1e3, "apply_us_in_solve": apply_in_solve_ms * 1e3,
                     "timing": "HIP events around 50 back-to-back launches of the PCG apply kernel",
                     "bytes_per_launch": apply_bytes},
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
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-copies comparison path")
    ap.add_argument("--no-tpfa", action="store_true", help="skip the cell-centred TPFA companion line")
    ap.add_argument("--optimizer", choices=("mma", "oc"), default="mma",
                    help="design update of the optimisation workloads (cube128_to_512_continuation, cube512_topopt)")
    ap.add_argument("--copies", choices=("bf16", "f32", "mixed"), default="bf16",
                    help="coefficient copies of the single-path workloads (interpolation, optimisation, 1024^3)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for the HBM counters)")
    ap.add_argument("--workload", default=None,
                    help="run a companion workload instead of the benchmark: cube128_grf8_c1e6, "
                         "cube256_grf16_paper_pair, cube128_to_512_continuation, cube512_paper_contrasts, "
                         "cube512_tpfa_paper_contrasts, cube256_adaptive_basis, cube128_to_512_tpfa_continuation, "
                         "cube256_grf16_contrast_sweep, cube512_topopt, cube512_grf32_warmstart, "
                         "cube1024_grf32_c1e6")
    ap.add_argument("--iterations", type=int, default=20, help="optimisation iterations (cube512_topopt)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path (sharding is described in the design "
              "notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload:
        run_workload(args.workload, args)
        return

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

    def run_path(opts, steps, warmup, tag, keep=None):
        s = pkg.Solver(n, timing=1, tune_cache=TUNE_CACHE, **opts)
        f = s.element_load(const=1.0)
        T = torch.empty_like(f)
        T_lo = torch.empty_like(f)
        recs = []
        for k in range(warmup + steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.setup(rho, KMIN, 1.0, 3, mask)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            T, info = s.solve(f, T, rtol=RTOL, maxit=1000, T_lo=T_lo)
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
        # the apply kernel alone, launched back to back on this set-up (the
        # in-solve events above also count each launch's dispatch gap)
        recs[-1]["apply_b2b_ms"] = s.time_apply(T, 50)
        if keep is not None:
            keep[tag] = (T + T_lo).cpu()
            if tag == "fp64":
                # reference for the solution errors: the FP64 path to 1e-12
                Tr_lo = torch.empty_like(f)
                Tr, ir = s.solve(f, rtol=1e-12, maxit=3000, T_lo=Tr_lo)
                keep["ref"] = (Tr + Tr_lo).cpu()
                keep["ref_info"] = dict(iterations=ir.iterations, rel_res=ir.rel_res, code=ir.code)
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

    sols = {}
    _log("mixed-precision path")
    mix = run_path(PATHS["mixed"], args.steps, args.warmup, "mixed", keep=sols)
    t_solve = float(np.mean([r["solve"] for r in mix]))
    t_step = float(np.mean([r["step"] for r in mix]))
    info = mix[-1]["info"]
    # dominant kernel: the PCG operator apply (one launch per iteration), timed
    # with HIP events on the solve stream: 50 back-to-back launches of the
    # PCG's apply kernel on the last set-up (msmg_time_apply), and, for
    # reference, per launch inside the timed solves (which adds each launch's
    # dispatch gap)
    apply_ms = float(mix[-1]["apply_b2b_ms"])
    apply_in_solve_ms = float(np.mean([r["info"]["apply_ms"] for r in mix]))
    nn, ne = (n + 1) ** 3, n ** 3
    apply_bytes = 16 * nn + 8 * ne + nn / 8  # p read, q written, the FP64 density read, mask bits
    achieved = apply_bytes / (apply_ms * 1e-3) / 1e9
    traffic = measured_traffic() if n == N else None

    # practical ceiling of the apply's access mix on this device: the same
    # bytes streamed once each without the stencil (msmg_stream_ceiling)
    ceiling = None
    try:
        import ctypes

        from paper_2410_06850_amd import _lib as L

        nn_e = (n + 1) ** 3 // 2 * 2
        xa = torch.ones(nn_e, dtype=torch.float64, device=dev)
        ka = torch.ones(n ** 3, dtype=torch.float64, device=dev)
        ya = torch.empty_like(xa)
        ms = ctypes.c_double()
        L.check(L.lib().msmg_stream_ceiling(ctypes.c_void_p(xa.data_ptr()), ctypes.c_void_p(ka.data_ptr()),
                                            ctypes.c_void_p(ya.data_ptr()), nn_e, n ** 3, 20, ctypes.byref(ms),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
                "msmg_stream_ceiling")
        cbytes = 8.0 * (2 * nn_e + n ** 3)
        cgbs = cbytes / (ms.value * 1e-3) / 1e9
        ceiling = {"kernel": "k_stream_ceiling (one coalesced read of x and k, one write of y)", "us": ms.value * 1e3,
                   "bytes": cbytes, "achieved": cgbs, "frac_of_peak": cgbs / HBM_PEAK_GBS,
                   "apply_frac_of_ceiling": achieved / cgbs}
        del xa, ka, ya
        torch.cuda.empty_cache()
    except Exception as e:  # the measurement aid is optional; the bench line stands without it
        _log(f"stream ceiling not measured: {e}")

    others = {}
    if not args.no_fp64:
        _log("FP64 path")
        others["fp64"] = summary(run_path(PATHS["fp64"], args.steps, args.warmup, "fp64", keep=sols))
    if not args.no_bf16:
        _log("BF16-copies path")
        others["bf16"] = summary(run_path(PATHS["bf16"], args.steps, args.warmup, "bf16", keep=sols))
    if not args.no_f32:
        _log("FP32-cycle path")
        others["f32cycle"] = summary(run_path(PATHS["f32cycle"], args.steps, args.warmup, "f32cycle", keep=sols))

    # solution errors of every path against the FP64 path and against the FP64
    # reference solved to 1e-12 (the one operator; differences are bounded by
    # cond(A) x the two residuals)
    errors = {}
    if "fp64" in sols:
        b64, ref = sols["fp64"], sols["ref"]
        for tag, T_ in sols.items():
            if tag in ("ref", "ref_info"):
                continue
            errors[tag] = {"vs_fp64": float(torch.linalg.norm(T_ - b64) / torch.linalg.norm(b64)),
                           "vs_fp64_rtol1e-12": float(torch.linalg.norm(T_ - ref) / torch.linalg.norm(ref))}
        errors["reference"] = sols["ref_info"]
    del sols

    def setup_report(recs, n):
        # set-up phases from HIP events inside the timed set-ups (options.timing);
        # the dense inversions (shifted coarse-coarse matrices, A_cc) with their
        # n^3 flops against the FP64 peak
        ph = np.mean([r["info"]["setup_phase_ms"] for r in recs], axis=0)
        dms = float(np.mean([r["info"]["setup_dense_ms"] for r in recs]))
        dgf = float(recs[-1]["info"]["setup_dense_gflop"])
        ncells = (n // 8) ** 3
        return {
            "ms": 1e3 * float(np.mean([r["setup"] for r in recs])),
            "phases_ms": {"local_spectral_problems": float(ph[0]), "galerkin_Ac": float(ph[1]),
                          "coarse_coarse_problems": float(ph[2]), "Acc_and_inverse": float(ph[3])},
            "local_problems_per_s": ncells / (float(ph[0]) * 1e-3) if ph[0] > 0 else None,
            "dense_inverses": {"ms": dms, "gflop": dgf, "tflops": dgf / dms if dms > 0 else None,
                               "peak_tflops": FP64_PEAK_TFLOPS,
                               "frac": dgf / dms / FP64_PEAK_TFLOPS if dms > 0 else None},
        }

    tpfa_line = None
    if not args.no_tpfa:
        _log("TPFA (cell-centred) path")
        tpfa_line = run_tpfa(pkg, rho, n, args.steps, args.warmup)

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
            "precision": ("FP64 PCG (double-double iterate) and FP64 cycle arithmetic; BF16 copy of k, FP32 copy of R_c, "
                          "FP32 Jacobi diagonal in the cycle; FP64 coarse levels"),
            "step": "set-up + PCG solve from zero + compliance sensitivity; value counts the solve only",
        },
        "iterations": info["iterations"],
        "rel_res": info["rel_res"],
        "solve_ms": 1e3 * t_solve,
        "setup_ms": 1e3 * float(np.mean([r["setup"] for r in mix])),
        "precond_us": 1e3 * float(np.mean([r["info"]["precond_ms"] for r in mix])),
        "setup": setup_report(mix, n),
        "paths": others,
        "solution_errors": errors,
        "roofline": {
            "kernel": "k_apply (PCG operator apply q = A p, FP64, difference form)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "apply_us": apply_ms * 1e3,
            "apply_us_in_solve": apply_in_solve_ms * 1e3,
            "timing": "HIP events around 50 back-to-back launches of the PCG apply kernel on the solve stream",
            "bytes_per_launch": apply_bytes,
            "ceiling": ceiling,
        },
        "tpfa": tpfa_line,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
