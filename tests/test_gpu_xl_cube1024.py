"""Full-size case: 1024^3 elements (1,076,848,600 free DOFs) on one GPU with the
lean layout and an FP32 density (GRF ell 32, contrast 1e6), solved cold to
true relative residual 1e-8, in the configuration bench.py's 1024^3 workload
runs.  The oracle cannot assemble this operator, so it checks sampled rows:
its node-by-node residual rows of the GPU solution against the GPU's own
operator rows, and the load rows against the GPU's load.

Part of the default GPU suite: about three minutes and 220 GB of device
memory (the file name sorts it after the faster GPU tests).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import q1

pytestmark = pytest.mark.gpu

N, KMIN, KMAX, P, RTOL = 1024, 1e-6, 1.0, 3, 1e-8


def _sample_nodes(g, mask, rng):
    free = np.flatnonzero(mask == 0)
    picks = [rng.choice(free, 20000, replace=False)]
    # every node of small boxes at the patch edge, a face, an edge and a corner
    for (i0, j0, k0) in ((N // 2 - N // 10 - 2, N // 2 - 2, 0), (0, N // 2, N // 2), (0, 0, N // 2), (N - 3, N - 3, N - 3)):
        i, j, k = np.meshgrid(np.arange(i0, i0 + 4), np.arange(j0, j0 + 4), np.arange(k0, k0 + 4), indexing="ij")
        ids = g.node_index(i.ravel(), j.ravel(), k.ravel())
        picks.append(ids[mask[ids] == 0])
    return np.unique(np.concatenate(picks))


def test_cube1024_sampled_rows_match_oracle():
    import paper_2410_06850_amd as pkg

    print("case cube1024 grf ell 32 contrast 1e6, lean layout, FP32 density, cold solve", flush=True)
    w = synth.grf_raw(N, 32, seed=0, dtype=np.float32)
    rho = synth.threshold_field(w, dtype=np.float32).ravel()
    del w
    mask = synth.dirichlet_patch_mask(N, N, N).ravel()
    s = pkg.Solver(N, vcycle_dtype=0, rho_v_dtype=2, basis_dtype=2, rho_storage=1, lean_memory=1)
    assert s.plan().device_bytes < 200e9
    s.setup(torch.from_numpy(rho).cuda(), KMIN, KMAX, P, torch.from_numpy(mask).cuda())
    f = s.element_load(const=1.0)
    T_lo = torch.empty_like(f)
    T, info = s.solve(f, rtol=RTOL, maxit=2000, T_lo=T_lo)
    print(f"  iterations {info.iterations} rel_res {info.rel_res:.3e} solve {info.solve_ms:.0f} ms", flush=True)
    assert info.code == 0 and info.rel_res <= RTOL
    y = s.apply(T)                   # A (T + T_lo) on free rows, masked form
    y.add_(s.apply(T_lo))
    g = q1.Grid(N)
    nodes = _sample_nodes(g, mask, np.random.default_rng(0))
    idx = torch.from_numpy(nodes).cuda()
    f_gpu, y_gpu = f[idx].cpu().numpy(), y[idx].cpu().numpy()
    del y
    # the load rows
    f_or = q1.element_load_rows(g, 1.0, nodes)
    assert np.allclose(f_gpu, f_or, rtol=1e-15, atol=0)
    # residual rows of the GPU solution, oracle vs GPU operator
    Th, Tl = T.cpu().numpy(), T_lo.cpu().numpy()
    r_or, absum = q1.residual_rows(g, rho, KMIN, KMAX, P, Th, f_or, nodes, T_lo=Tl)
    r_gpu = f_gpu - y_gpu
    err = np.abs(r_or - r_gpu)
    print(f"  {nodes.size} rows: max |r_oracle - r_gpu| / (sum |terms| + |f|) = {np.max(err / (absum + np.abs(f_or))):.2e}",
          flush=True)
    assert np.all(err <= 1e-12 * (absum + np.abs(f_or)))
    # the sampled rows estimate the true relative residual the GPU reports
    b_norm = np.sqrt(float((f[torch.from_numpy(mask == 0).cuda()] ** 2).sum()))
    est = np.sqrt(np.mean(r_or ** 2) * float((mask == 0).sum())) / b_norm
    print(f"  sampled-row estimate of the relative residual {est:.2e} (reported {info.rel_res:.2e})", flush=True)
    assert est <= 10 * RTOL
