"""Pins of the oracle's Neumann model problem (Sec. 3.1, Eq. Laplace): the mirrored-ghost
step against the operator assembled by hand, its spectrum against the DCT-II closed form,
and whole SRJ and Jacobi solves against the exact modal trajectory (CPU only)."""
import math

import numpy as np
import pytest

from oracle import neumann as NE
from oracle import schedule as S
from oracle import sweeps


def neumann_matrix_by_hand(n_xyz, h=None):
    """A = dg I - (weighted neighbour couplings), each missing neighbour replaced by the cell
    itself (its coupling moves onto the diagonal): assembled point by point."""
    nd = len(n_xyz)
    wt = sweeps.axis_weights(h if h is not None else 1.0, nd)
    a = (1.0, wt[0], wt[1])
    n = int(np.prod(n_xyz))
    A = np.zeros((n, n))

    def idx(p):
        k = 0
        for ax in reversed(range(nd)):
            k = k * n_xyz[ax] + p[ax]
        return k

    for flat in range(n):
        p, r = [], flat
        for ax in range(nd):
            p.append(r % n_xyz[ax])
            r //= n_xyz[ax]
        A[flat, flat] += wt[2]
        for ax in range(nd):
            for d in (-1, 1):
                qq = list(p)
                qq[ax] += d
                if not 0 <= qq[ax] < n_xyz[ax]:
                    qq[ax] = p[ax]
                A[flat, idx(qq)] -= a[ax]
    return A


@pytest.mark.parametrize("n_xyz,h", [((5, 4), None), ((6, 3), (0.1, 0.25)), ((3, 4, 2), None),
                                      ((4, 2, 3), (0.2, 0.1, 0.3))])
def test_neumann_step_and_residual_match_matrix_form(n_xyz, h):
    nd = len(n_xyz)
    rng = np.random.default_rng(31)
    full = tuple(x + 2 for x in reversed(n_xyz))
    u = rng.uniform(-1, 1, size=full)
    b = rng.uniform(-1, 1, size=full)
    wt = sweeps.axis_weights(h if h is not None else 1.0, nd)
    A = neumann_matrix_by_hand(n_xyz, h)
    inner = tuple(slice(1, -1) for _ in range(nd))
    x = u[inner].ravel()
    c = 2.5 / wt[2]
    out = NE.sweep(u, b, c, wt)
    ref = x + c * (b[inner].ravel() - A @ x)
    assert np.max(np.abs(out[inner].ravel() - ref)) <= 1e-14 * np.max(np.abs(ref))
    ring = np.ones(full, bool)
    ring[inner] = False
    assert np.array_equal(out[ring], u[ring])
    r, r2, rmax = NE.residual(u, b, wt)
    rr = b[inner].ravel() - A @ x
    assert np.max(np.abs(r[inner].ravel() - rr)) <= 1e-14 * np.max(np.abs(rr))
    assert math.isclose(r2, float(np.sum(rr * rr)), rel_tol=1e-13) and math.isclose(rmax, float(np.max(np.abs(rr))),
                                                                                    rel_tol=1e-13)
    # the spectrum is the DCT-II closed form; its smallest nonzero symbol is kappa_min
    ev = np.sort(np.linalg.eigvalsh(A))
    lam = np.sort(NE.eigenvalues(tuple(reversed(n_xyz)), wt).ravel())
    np.testing.assert_allclose(ev, lam, atol=1e-12)
    assert abs(ev[0]) < 1e-12 and math.isclose(ev[1] / wt[2], NE.kappa_min(n_xyz, h), rel_tol=1e-12)


def test_neumann_kappa_min_is_eq_boundaries():
    # equal spacings: (2/d) sin^2(pi / 2N) with N the largest cell count (Eq. boundaries1D3D)
    assert NE.kappa_min((64, 64)) == S.kappa_min_neumann(64)
    assert math.isclose(NE.kappa_min((40, 64)), S.kappa_min_neumann(64), rel_tol=1e-15)
    assert math.isclose(NE.kappa_min((30, 30, 30)), S.kappa_min_neumann(30, 3), rel_tol=1e-15)


@pytest.mark.parametrize("P", [2, 3, 5])
def test_neumann_srj_solve_follows_modal_trajectory(P):
    """The Laplace problem of Eq. Laplace from a random start on 48^2 cells: the SRJ solve
    stops at the cycle the DCT-mode trajectory predicts, with the relres it predicts."""
    N = 48
    rng = np.random.default_rng(P)
    u0 = rng.uniform(-1, 1, (N + 2, N + 2))
    f = np.zeros_like(u0)
    km = S.kappa_min_neumann(N)
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    res = NE.solve(u0, f, 1.0 / N, np.asarray(o["w"])[seq], 1e-10, 10 ** 7, history=True)
    M = int(np.sum(q))
    m = NE.cycles_to(u0, f, o["w"], q, 1e-10)
    assert res["status"] == "ok" and res["sweeps"] == m * M
    pred = NE.predicted_relres(u0, f, o["w"], q, m)
    np.testing.assert_allclose(res["history"], pred, rtol=1e-6, atol=1e-15)
    # the constant mode (the mean) is invariant: the limit is the mean of the start
    inner = (slice(1, -1), slice(1, -1))
    assert abs(float(np.mean(res["u"][inner])) - float(np.mean(u0[inner]))) <= 1e-12


def test_neumann_jacobi_follows_modal_trajectory():
    N = 24
    rng = np.random.default_rng(7)
    u0 = rng.uniform(-1, 1, (N + 2, N + 2))
    f = np.zeros_like(u0)
    res = NE.solve(u0, f, 1.0 / N, [1.0], 1e-8, 10 ** 6)
    assert res["status"] == "ok" and res["sweeps"] == NE.cycles_to(u0, f, [1.0], [1], 1e-8)
