"""Differentiable solve: adjoint SRJ gradients against the oracle's dense-solve gradient and
against central finite differences (L is quadratic in (f, g), so central differences carry no
truncation error; what remains is the solve tolerance and rounding)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as OA
from oracle import schedule as S
from paper_1511_04292_amd import srj, workloads
from paper_1511_04292_amd.autograd import srj_solve_diff

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def oracle_plan(n, h, P):
    km = S.kappa_min_dirichlet(n)
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    return srj.srj_plan(n, h, omega=o["w"], q=q, sequence=S.order_balanced(o["w"], q, km))


def problem(n, seed):
    rng = np.random.default_rng(seed)
    full = tuple(x + 2 for x in reversed(n))
    g = workloads.random_ring(full, rng)
    f = np.zeros(full)
    f[tuple(slice(1, -1) for _ in full)] = rng.standard_normal(tuple(reversed(n)))
    ut = rng.standard_normal(full) * 0.1
    return f, g, ut


def loss_t(u, ut):
    inner = tuple(slice(1, -1) for _ in range(u.dim()))
    return 0.5 * ((u - ut)[inner] ** 2).sum()


@pytest.mark.parametrize("n,P", [((32, 32), 3), ((27, 20), 4), ((7, 5, 6), 3)])
def test_adjoint_matches_dense_gradient(n, P):
    h = 1.0 / (max(n) + 1)
    f, g, ut = problem(n, 11)
    plan = oracle_plan(n, h, P)
    ft = dev(f).requires_grad_(True)
    gt = dev(g).requires_grad_(True)
    u = srj_solve_diff(ft, gt, plan, tol=1e-13, tol_backward=1e-13)
    L = loss_t(u, dev(ut))
    L.backward()
    df_ref, dg_ref = OA.grad_dense(f, g, ut, h)
    u_ref = OA.forward_dense(f, g, h)
    assert abs(float(L) - OA.loss(u_ref, ut)) <= 1e-9 * OA.loss(u_ref, ut)
    df = ft.grad.cpu().numpy()
    dg = gt.grad.cpu().numpy()
    assert np.max(np.abs(df - df_ref)) <= 1e-9 * np.max(np.abs(df_ref))
    assert np.max(np.abs(dg - dg_ref)) <= 1e-9 * np.max(np.abs(dg_ref))
    # structure: df zero on the ring, dg zero inside and at the 2D corners
    inner = tuple(slice(1, -1) for _ in n)
    ring = np.ones(df.shape, bool)
    ring[inner] = False
    assert not np.any(df[ring]) and not np.any(dg[~ring])
    if len(n) == 2:
        assert dg[0, 0] == dg[0, -1] == dg[-1, 0] == dg[-1, -1] == 0.0


def test_adjoint_central_differences():
    n = (129, 96)
    h = 1.0 / 130
    f, g, ut = problem(n, 12)
    plan = srj.srj_plan(n, h, P=5)
    ft = dev(f).requires_grad_(True)
    gt = dev(g).requires_grad_(True)
    L = loss_t(srj_solve_diff(ft, gt, plan, tol=1e-13, tol_backward=1e-13), dev(ut))
    L.backward()
    df, dg = ft.grad, gt.grad
    rng = np.random.default_rng(2)
    inner = (slice(1, -1), slice(1, -1))
    for _ in range(6):
        vf = np.zeros_like(f)
        vf[inner] = rng.standard_normal((96, 129))
        vg = workloads.random_ring(f.shape, rng)
        eps = 1e-2
        with torch.no_grad():
            lp = float(loss_t(srj_solve_diff(dev(f + eps * vf), dev(g + eps * vg), plan, tol=1e-13), dev(ut)))
            lm = float(loss_t(srj_solve_diff(dev(f - eps * vf), dev(g - eps * vg), plan, tol=1e-13), dev(ut)))
        fd = (lp - lm) / (2 * eps)
        an = float((df * dev(vf)).sum() + (dg * dev(vg)).sum())
        assert abs(fd - an) <= 1e-7 * abs(an) + 1e-12, (fd, an)


def test_ring_gradient_passes_through():
    n = (30, 22)
    h = 1.0 / 31
    f, g, _ = problem(n, 13)
    plan = srj.srj_plan(n, h, P=3)
    gt = dev(g).requires_grad_(True)
    u = srj_solve_diff(dev(f), gt, plan, tol=1e-12)
    w = torch.zeros_like(u)
    w[0, 5] = 2.0  # loss reads one ring value of u only
    (u * w).sum().backward()
    expect = np.zeros_like(g)
    expect[0, 5] = 2.0
    assert np.array_equal(gt.grad.cpu().numpy(), expect)
