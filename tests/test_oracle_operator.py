"""Pins of the oracle's variable-coefficient operator with a mask (Sec. 5.3): the scaled step
against the system assembled point by point, masked solves against a sparse direct solve, the
Poisson coefficients against the Poisson sweep, and the Grad-Shafranov test A solution against
its analytic dipole (CPU only)."""
import math

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

from oracle import operator as OP
from oracle import schedule as S
from oracle import spectral, sweeps
from paper_1511_04292_amd import workloads


def random_operator(shape, seed, masked=True):
    """Diagonally dominant random coefficients (a_P = 1.1 sum a_nb), random fixed values on
    the ring, and a random mask of about a fifth of the interior."""
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
        ring = np.ones(shape, bool)
        ring[tuple(slice(1, -1) for _ in shape)] = False
        mask[ring] = 0
    return coef, u, f, mask


@pytest.mark.parametrize("shape", [(9, 12), (5, 6, 7)])
def test_scaled_step_matches_assembled_system(shape):
    coef, u, f, mask = random_operator(shape, 1)
    A, rhs, free = OP.dense_system(coef, f, u, mask)
    wts, bs = OP.scale(coef, f)
    omega = 1.7
    out = OP.sweep(u, wts, bs, omega, mask)
    x = u[free]
    d = coef[0][free]
    ref = x + omega * (rhs - A @ x) / d
    assert np.max(np.abs(out[free] - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert np.array_equal(out[~free], u[~free])
    t, t2, tmax = OP.residual(u, wts, bs, mask)
    tt = (rhs - A @ x) / d
    assert np.max(np.abs(t[free] - tt)) <= 1e-14 * np.max(np.abs(tt)) and not np.any(t[~free])
    assert math.isclose(t2, float(np.sum(tt * tt)), rel_tol=1e-13)


def test_masked_solve_matches_sparse_direct_solve():
    shape = (22, 31)
    coef, u, f, mask = random_operator(shape, 2)
    A, rhs, free = OP.dense_system(coef, f, u, mask)
    exact = scipy.sparse.linalg.spsolve(scipy.sparse.csr_matrix(A), rhs)
    km = 0.01
    o = S.optimal(4, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    res = OP.solve(u, f, coef, np.asarray(o["w"])[seq], 1e-12, 10 ** 6, mask=mask)
    assert res["status"] == "ok" and res["relres"] <= 1e-12
    assert np.max(np.abs(res["u"][free] - exact)) <= 1e-9 * np.max(np.abs(exact))
    assert np.array_equal(res["u"][~free], u[~free])


def test_poisson_coefficients_give_the_poisson_solution():
    """a_P = 4, a_nb = 1 and f = h^2 f_Poisson: the operator route reaches the exact discrete
    Poisson solution (DST), and a single scaled step equals the Poisson step to rounding."""
    n = 40
    wl = workloads.small_2d(n, seed=4)
    shape = wl["f"].shape
    coef = np.ones((5,) + shape)
    coef[0] = 4.0
    b = sweeps.rhs(wl["f"], wl["h"])
    wts, bs = OP.scale(coef, b)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, shape)
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
    one = OP.sweep(u, wts, bs, 3.0)
    ref = sweeps.sweep(u, b, 3.0 / 4.0)
    assert np.max(np.abs(one - ref)) <= 4e-15 * np.max(np.abs(ref))
    km = S.kappa_min_dirichlet((n, n))
    o = S.optimal(3, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    res = OP.solve(wl["u0"], b, coef, np.asarray(o["w"])[seq], 1e-12, 10 ** 6)
    us = spectral.exact_solve(wl["u0"], b)
    assert np.max(np.abs(res["u"] - us)) <= 1e-8 * np.max(np.abs(us))


def test_grad_shafranov_test_a_dipole():
    """Sec. 5.3 test A with C = 0 on the paper's 300 x 300 points: the discrete solution (sparse
    direct solve of the assembled system) differs from the analytic dipole sin^2(th)/r by about
    9/N^2, as the paper reports (8.5e-5)."""
    wl = workloads.grad_shafranov(298, 0.0, "A")
    A, rhs, free = OP.dense_system_sparse(wl["coef"], wl["f"], wl["u0"], wl["mask"])
    x = scipy.sparse.linalg.spsolve(A.tocsc(), rhs)
    err = float(np.max(np.abs(x - wl["u_exact"][free])))
    assert 5e-5 < err < 9.0 / 300 ** 2, err


def test_spherical_poisson_discretisation_is_second_order():
    """Sec. 5.2's axisymmetric Poisson test: the discrete system (centre folded, axis ghosts,
    exact exterior data at r = 1 + dr/2), solved directly, approaches the series solution at
    second order, and its Jacobi-scaled operator is diagonally dominant (Jacobi symbols in
    [0, 2])."""
    import scipy.sparse.linalg as spla

    errs = []
    for N in (16, 32, 64):
        wl = workloads.spherical_poisson_2d(N)
        c = wl["coef"]
        inner = (slice(1, -1), slice(1, -1))
        assert np.all(c[0][inner] + 1e-12 * c[0][inner] >= c[1][inner] + c[2][inner] + c[3][inner] + c[4][inner])
        assert np.all(c[1:][(slice(None),) + inner] >= 0)
        A, rhs, free = OP.dense_system_sparse(c, wl["f"], wl["u0"])
        u = wl["u0"].copy()
        u[free] = spla.spsolve(A.tocsr(), rhs)
        errs.append(np.max(np.abs(u - wl["u_exact"])[inner]))
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2, errs
    # the series solution is continuous at r = 1 and its source vanishes there
    s, u = workloads.spherical_series(np.array([1.0 - 1e-9, 1.0 + 1e-9]), np.array([0.4, 0.4]))
    assert abs(u[0] - u[1]) < 1e-8 and abs(s[0]) < 1e-7
