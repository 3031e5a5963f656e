"""The allocation-free residual entry point (srj_residual_static) against the plan-based
srj_residual, through the C ABI: the same norms and residual field, bit for bit, on two calls
in a row on one GPU (the second on a smaller grid, so stale scratch contents from the first
call would show), in 2D and 3D; grids beyond its scratch are rejected before any launch."""
import numpy as np
import pytest
import torch

from paper_1511_04292_amd import srj, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(n, seed):
    full = tuple(x + 2 for x in reversed(n))
    u = workloads.random_state(full, seed)
    f = workloads.random_state(full, seed + 1)
    return torch.from_numpy(u).to(DEV), torch.from_numpy(f).to(DEV)


def _plan_based(n, h, u, f):
    p = srj.srj_plan(n, h, omega=[1.0], q=[1])
    r = torch.full_like(u, 7.0)
    nr = srj.srj_residual(p, u, f, r)
    return np.array([nr["l2"], nr["linf"], nr["source_l2"], nr["relres"]]), r.cpu().numpy()


@pytest.mark.parametrize("sizes", [[(300, 257), (64, 45)], [(33, 20, 17), (9, 5, 4)]])
def test_static_residual_matches_plan_residual(sizes):
    norms = torch.zeros(4, dtype=torch.float64, device=DEV)
    for k, n in enumerate(sizes):
        h = 1.0 / (max(n) + 1)
        u, f = _case(n, 40 + k)
        r = torch.full_like(u, 7.0)
        srj.srj_residual_static(n, h, u, f, norms, r)
        torch.cuda.synchronize()
        got = norms.cpu().numpy().copy()
        ref, rref = _plan_based(n, h, u, f)
        assert np.array_equal(got, ref), (n, got, ref)
        assert np.array_equal(r.cpu().numpy(), rref), n
        # norms only, no residual field
        norms.fill_(-1.0)
        srj.srj_residual_static(n, h, u, f, norms)
        torch.cuda.synchronize()
        assert np.array_equal(norms.cpu().numpy(), ref)


def test_static_residual_rejects_grids_beyond_its_scratch():
    u = torch.zeros(4, dtype=torch.float64, device=DEV)
    g = srj._Grid()
    g.ndim = 2
    g.n[0], g.n[1] = 4, 600000  # 600000 rows > 524288 the scratch holds
    g.h[0] = g.h[1] = 1e-6
    g.dtype = 0
    import ctypes

    st = srj.lib().srj_residual_static(ctypes.byref(g), ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                        None, ctypes.c_void_p(u.data_ptr()), None)
    assert st == 1
    assert b"static scratch" in srj.lib().srj_last_error()
