"""The Neumann model problem of Sec. 3.1 (Eq. Laplace) on the GPU, through the C ABI, against
the oracle: mirrored-ghost sweeps bit for bit (2D and 3D, equal and unequal spacings),
residuals, the plan's spectral interval, and whole SRJ and Jacobi solves (same stopping sweep,
same iterate, and the cycle the exact DCT-mode trajectory predicts)."""
import math

import numpy as np
import pytest
import torch

from oracle import neumann as NE
from oracle import schedule as S
from oracle import sweeps
from paper_1511_04292_amd import srj

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sched(P, km):
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    return o["w"], q, S.order_balanced(o["w"], q, km)


@pytest.mark.parametrize("n,h", [((70, 45), None), ((2, 9), None), ((64, 33), (1.0 / 64, 1.0 / 20)),
                                 ((20, 17, 13), None), ((9, 12, 5), (0.1, 0.2, 0.05))])
def test_neumann_sweeps_bitwise(n, h):
    nd = len(n)
    hh = h if h is not None else 1.0 / max(n)
    rng = np.random.default_rng(4)
    full = tuple(x + 2 for x in reversed(n))
    u = rng.uniform(-1, 1, full)
    f = rng.uniform(-1, 1, full)
    wt = sweeps.axis_weights(hh, nd)
    km = NE.kappa_min(n, h)
    w, q, seq = sched(3, km)
    p = srj.srj_plan(n, hh, omega=w, q=q, sequence=seq, bc="neumann")
    d = srj.srj_plan_describe(p)
    assert d["fused_sweeps"] == (8 if nd == 2 else 0)  # 2D: tiles in LDS, 3D: unfused
    nsw = len(seq) + 5
    c = sweeps.coefficients(np.asarray(w)[seq], nd, wt)
    ref = NE.run(u, sweeps.rhs(f, hh), c, nsw, k0=1, wt=wt)
    inner = tuple(slice(1, -1) for _ in range(nd))
    for fuse in ((8, 5, 0) if nd == 2 else (0,)):
        srj.srj_plan_set_fusion(p, fuse)
        ug = dev(u)
        srj.srj_sweeps(p, ug, dev(f), 1, nsw)
        got = host(ug)
        assert np.array_equal(got[inner], ref[inner]), fuse
    # residual norms and field
    r = torch.zeros_like(ug)
    nr = srj.srj_residual(p, dev(u), dev(f), r)
    rf, r2, rmax = NE.residual(u, sweeps.rhs(f, hh), wt)
    assert math.isclose(nr["l2"], math.sqrt(r2), rel_tol=1e-12) and nr["linf"] == rmax
    assert np.array_equal(host(r), rf)
    # the plan's default interval starts at the smallest nonzero symbol
    p2 = srj.srj_plan(n, hh, P=2, bc="neumann")
    assert math.isclose(srj.srj_plan_describe(p2)["kappa_min"], km, rel_tol=1e-13)


@pytest.mark.parametrize("P", [2, 4, 5])
def test_neumann_laplace_solve_bitwise(P):
    """Eq. Laplace on 96^2 cells from a random start: the GPU solve stops where the oracle's
    does, at the cycle the DCT-mode trajectory predicts, with the same iterate."""
    N = 96
    rng = np.random.default_rng(10 + P)
    u0 = rng.uniform(-1, 1, (N + 2, N + 2))
    f = np.zeros_like(u0)
    km = S.kappa_min_neumann(N)
    w, q, seq = sched(P, km)
    ref = NE.solve(u0, f, 1.0 / N, np.asarray(w)[seq], 1e-10, 10 ** 7)
    p = srj.srj_plan((N, N), 1.0 / N, omega=w, q=q, sequence=seq, bc="neumann")
    ug = dev(u0)
    info = srj.srj_solve(p, ug, dev(f), 1e-10, 10 ** 7)
    assert info["status"] == "ok" and info["sweeps"] == ref["sweeps"]
    assert info["sweeps"] == NE.cycles_to(u0, f, w, q, 1e-10) * int(np.sum(q))
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
    inner = (slice(1, -1), slice(1, -1))
    assert np.array_equal(host(ug)[inner], ref["u"][inner])


def test_neumann_jacobi_and_refusals():
    N = 24
    rng = np.random.default_rng(3)
    u0 = rng.uniform(-1, 1, (N + 2, N + 2))
    f = np.zeros_like(u0)
    ref = NE.solve(u0, f, 1.0 / N, [1.0], 1e-8, 10 ** 6)
    p = srj.srj_plan((N, N), 1.0 / N, omega=[1.0], q=[1], bc="neumann")
    ug = dev(u0)
    info = srj.srj_solve(p, ug, dev(f), 1e-8, 10 ** 6)
    assert info["sweeps"] == ref["sweeps"]
    assert np.array_equal(host(ug)[1:-1, 1:-1], ref["u"][1:-1, 1:-1])
    # a state with zero residual (a constant) is returned unchanged
    c = np.full_like(u0, 0.25)
    ug = dev(c)
    info = srj.srj_solve(p, ug, dev(f), 1e-8, 10 ** 6)
    assert info["sweeps"] == 0 and torch.equal(ug, dev(c))
    with pytest.raises(srj.SrjError):
        srj.srj_plan((N, N), 1.0 / N, omega=[1.0], q=[1], bc="neumann", dtype="f32")
    with pytest.raises(srj.SrjError):
        srj.srj_plan_set_fusion(p, 9)
    with pytest.raises(srj.SrjError):
        srj.srj_solve_ir(p, dev(u0), dev(f), 1e-8, 1, 10)
