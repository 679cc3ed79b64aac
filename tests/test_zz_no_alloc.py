"""The allocation-free OC update (msmg_oc_update_noalloc) against the handle's
msmg_oc_update: the same kernels on the same grid, so x_new and the multiplier
agree bitwise, on two calls in a row (the second on a smaller design, which
reuses the device's scratch array left by the first)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _design(n, seed):
    rng = np.random.default_rng(seed)
    ne = n ** 3
    x = np.clip(0.3 + 0.2 * rng.standard_normal(ne), 1e-3, 1.0)
    dc = -np.exp(rng.standard_normal(ne))
    dv = np.ones(ne)
    return [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (x, dc, dv)]


def test_oc_update_noalloc_matches_handle_update():
    import paper_2410_06850_amd as pkg
    from paper_2410_06850_amd import _lib as L

    for n, seed in ((24, 1), (10, 2)):
        print(f"case oc-noalloc n={n} seed={seed}", flush=True)
        x, dc, dv = _design(n, seed)
        s = pkg.Solver(n, H=2, sd=2)
        want, lam_w = s.oc_update(x, dc, dv, 0.3, move=0.2, eta=0.5, x_min=1e-3)
        got = torch.empty_like(x)
        lam = torch.empty((), dtype=torch.float64, device="cuda")
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        code = L.lib().msmg_oc_update_noalloc(n, n, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(dc.data_ptr()),
                                              ctypes.c_void_p(dv.data_ptr()), 0.3, 0.2, 0.5, 1e-3,
                                              ctypes.c_void_p(got.data_ptr()), ctypes.c_void_p(lam.data_ptr()), stream)
        assert code == 0, L.last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        assert float(lam) == float(lam_w)
        assert abs(float(got.sum()) - 0.3 * n ** 3) <= 1e-6 * n ** 3
        del s
    # a design above the stated maximum is rejected before any launch
    code = L.lib().msmg_oc_update_noalloc(1 << 14, 1 << 14, 1 << 14, ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(dc.data_ptr()), ctypes.c_void_p(dv.data_ptr()), 0.3, 0.2,
                                          0.5, 1e-3, ctypes.c_void_p(got.data_ptr()), None, stream)
    assert code == L.MSMG_EINVAL and "at most" in L.last_error()
