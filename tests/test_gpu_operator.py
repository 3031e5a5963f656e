"""Variable-coefficient operators with a mask (srj_plan_operator; Sec. 5.3's Grad-Shafranov
operator and masked region) on the GPU, through the C ABI, against the oracle: scaled sweeps
and residuals bit for bit (2D and 3D, with and without a mask), whole solves, and the paper's
two Grad-Shafranov tests on its 300 x 300 grid with the P = 14, N = 300 scheme."""
import math

import numpy as np
import pytest
import torch

from oracle import operator as OP
from oracle import schedule as S
from paper_1511_04292_amd import srj, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def random_operator(shape, seed, masked):
    rng = np.random.default_rng(seed)
    nd = len(shape)
    coef = np.zeros((2 * nd + 1,) + shape)
    coef[1:] = rng.uniform(0.2, 1.0, (2 * nd,) + shape)
    coef[0] = 1.1 * coef[1:].sum(axis=0)
    u = rng.uniform(-1, 1, shape)
    f = rng.uniform(-1, 1, shape)
    mask = None
    if masked:
        mask = (rng.uniform(size=shape) < 0.2).astype(np.uint8)
    return coef, u, f, mask


def sched(P, km):
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    return o["w"], q, S.order_balanced(o["w"], q, km)


@pytest.mark.parametrize("n", [(70, 33), (5, 9), (21, 13, 17)])
@pytest.mark.parametrize("masked", [False, True])
def test_operator_sweeps_and_residual_bitwise(n, masked):
    shape = tuple(x + 2 for x in reversed(n))
    coef, u, f, mask = random_operator(shape, 3, masked)
    w, q, seq = sched(3, 0.01)
    p = srj.srj_plan_operator(n, dev(coef), dev(mask, torch.uint8) if masked else None, omega=w, q=q,
                              sequence=seq, kappa_min=0.01)
    nd = len(n)
    assert srj.srj_plan_describe(p)["fused_sweeps"] == (8 if nd == 2 else 0)  # 2D: tiles in LDS
    nsw = len(seq) + 4
    wts, bs = OP.scale(coef, f)
    ref = OP.run(u, wts, bs, np.asarray(w)[seq], nsw, k0=2, mask=mask)
    for fuse in ((8, 3, 0) if nd == 2 else (0,)):
        srj.srj_plan_set_fusion(p, fuse)
        ug = dev(u)
        srj.srj_sweeps(p, ug, dev(f), 2, nsw)
        assert np.array_equal(ug.cpu().numpy(), ref), fuse
    r = torch.zeros_like(ug)
    nr = srj.srj_residual(p, dev(u), dev(f), r)
    t, t2, tmax = OP.residual(u, wts, bs, mask)
    assert np.array_equal(r.cpu().numpy(), t)
    assert math.isclose(nr["l2"], math.sqrt(t2), rel_tol=1e-12) and nr["linf"] == tmax
    with pytest.raises(srj.SrjError):
        srj.srj_plan_set_fusion(p, 9 if nd == 2 else 2)
    with pytest.raises(srj.SrjError):
        srj.srj_solve_ir(p, dev(u), dev(f), 1e-8, 1, 5)


@pytest.mark.parametrize("test,C", [("A", 0.0), ("A", 0.2), ("B", 0.0), ("B", 1.0)])
def test_grad_shafranov_solves_bitwise(test, C):
    """Sec. 5.3 on its 300 x 300 points with the P = 14, N = 300 scheme, to relres 1e-12: the
    GPU stops where the oracle does with the same iterate; test A at C = 0 lies within 9/N^2
    of the dipole sin^2(th)/r."""
    wl = workloads.grad_shafranov(298, C, test)
    km = S.kappa_min_neumann(300)
    w, q, seq = sched(14, km)
    ref = OP.solve(wl["u0"], wl["f"], wl["coef"], np.asarray(w)[seq], 1e-12, 10 ** 6, mask=wl["mask"])
    mask = dev(wl["mask"], torch.uint8) if wl["mask"] is not None else None
    p = srj.srj_plan_operator(wl["n"], dev(wl["coef"]), mask, omega=w, q=q, sequence=seq, n_eff=300)
    ug = dev(wl["u0"])
    info = srj.srj_solve(p, ug, dev(wl["f"]), 1e-12, 10 ** 6)
    assert ref["status"] == "ok" and info["status"] == "ok"
    assert info["sweeps"] == ref["sweeps"]
    assert abs(info["relres"] - ref["relres"]) <= 1e-10 * ref["relres"]
    got = ug.cpu().numpy()
    assert np.array_equal(got, ref["u"])
    if test == "A" and C == 0.0:
        assert np.max(np.abs(got - wl["u_exact"])) < 9.0 / 300 ** 2
    # the product planner's scheme for the same row solves it too
    p2 = srj.srj_plan_operator(wl["n"], dev(wl["coef"]), mask, P=14, n_eff=300)
    ug2 = dev(wl["u0"])
    info2 = srj.srj_solve(p2, ug2, dev(wl["f"]), 1e-12, 10 ** 6)
    assert info2["status"] == "ok" and info2["sweeps"] == info["sweeps"]


def test_operator_plan_refusals():
    n = (8, 8)
    shape = (10, 10)
    coef, u, f, _ = random_operator(shape, 9, False)
    with pytest.raises(srj.SrjError):  # no interval for an optimised schedule
        srj.srj_plan_operator(n, dev(coef), None, P=3)
    with pytest.raises(TypeError):
        srj.srj_plan_operator(n, dev(coef[:4]), None, P=3, kappa_min=0.01)


@pytest.mark.parametrize("start", ["zero", "realistic"])
def test_spherical_poisson_solves_bitwise(start):
    """Sec. 5.2's Poisson equation in spherical coordinates (axisymmetric, r^2-scaled, 48 x 48
    cells) from a zero start and from the paper's warm start (the exact solution with 1/N
    relative noise): the GPU stops where the oracle does with the same iterate, within the
    discretisation error of the series solution; the warm start needs fewer sweeps."""
    N = 48
    wl = workloads.spherical_poisson_2d(N, start=start, seed=4)
    km = S.kappa_min_neumann(N)
    w, q, seq = sched(6, km)
    ref = OP.solve(wl["u0"], wl["f"], wl["coef"], np.asarray(w)[seq], 1e-10, 10 ** 6)
    p = srj.srj_plan_operator(wl["n"], dev(wl["coef"]), None, omega=w, q=q, sequence=seq, n_eff=N)
    ug = dev(wl["u0"])
    info = srj.srj_solve(p, ug, dev(wl["f"]), 1e-10, 10 ** 6)
    assert ref["status"] == "ok" and info["status"] == "ok"
    assert info["sweeps"] == ref["sweeps"]
    got = ug.cpu().numpy()
    assert np.array_equal(got, ref["u"])
    inner = (slice(1, -1), slice(1, -1))
    assert np.max(np.abs(got - wl["u_exact"])[inner]) < 1.5 * 0.00252 * (16 / N) ** 2
    if start == "realistic":
        cold = OP.solve(workloads.spherical_poisson_2d(N)["u0"], wl["f"], wl["coef"], np.asarray(w)[seq], 1e-10,
                        10 ** 6)
        assert info["sweeps"] < cold["sweeps"]
