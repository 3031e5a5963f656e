"""The Neumann model problem of Sec. 3.1 (Eq. Laplace) -- oracle side, test infrastructure.

The Laplace (or a compatible Poisson) problem with homogeneous Neumann boundaries on a
cell-centred grid of N_i cells per axis: the ring of the arrays holds ghost cells that mirror
the adjacent cell, so across the boundary a cell's neighbour is the cell itself.  One
weighted-Jacobi step (Eq. 2nd-order_CD) is the Dirichlet step of ``sweeps`` with those
neighbours (same association and axis weights); the ring is never read.

The operator is singular: constants are in its null space, and the scheme leaves the
constant part of the error unchanged (G(0) = 1).  The residual reference is therefore the
initial residual: relres_k = ||r_k||_2 / ||r_0||_2, checked at cycle ends.  The type-II DCT
diagonalises the operator (Sec. 3.1's kappa(k_x, k_y) = sin^2(k_x pi / 2N_x) + sin^2(k_y pi / 2N_y),
k_i = 0..N_i - 1), which pins the sweeps through the exact modal trajectory.
"""
import ctypes

import numpy as np
import scipy.fft

from ._clib import lib
from .sweeps import _c64, _dims, _p, _wt, axis_weights, coefficients, rhs


def sweep(u, b, c, wt=None):
    """One weighted-Jacobi step with mirrored boundary neighbours."""
    u = _c64(u)
    b = _c64(b)
    w = _wt(wt, u.ndim)
    out = u.copy()
    d = _dims(u)
    if u.ndim == 2:
        lib().or_sweep2d_neu(d[0], d[1], _p(u), _p(b), _p(w), float(c), _p(out))
    else:
        lib().or_sweep3d_neu(d[0], d[1], d[2], _p(u), _p(b), _p(w), float(c), _p(out))
    return out


def run(u, b, c_seq, nsweeps, k0=0, wt=None):
    """nsweeps scheduled steps; step s uses c_seq[(k0 + s) mod M] (Sec. 2)."""
    u = _c64(u).copy()
    M = len(c_seq)
    for s in range(nsweeps):
        u = sweep(u, b, c_seq[(k0 + s) % M], wt)
    return u


def residual(u, b, wt=None):
    """(r field with a zero ring, sum r^2, max |r|) of r = b - A u."""
    u = _c64(u)
    b = _c64(b)
    w = _wt(wt, u.ndim)
    d = _dims(u)
    nz = d[2] if u.ndim == 3 else 1
    r = np.empty_like(u)
    out = np.zeros(2)
    rs = np.zeros(d[1] * nz)
    rm = np.zeros(d[1] * nz)
    lib().or_residual_neu(d[0], d[1], nz, ctypes.c_int(u.ndim), _p(u), _p(b), _p(w), _p(r), _p(out), _p(rs), _p(rm))
    return r, float(out[0]), float(out[1])


def solve(u0, f, h, omega_sequence, tol, max_sweeps, history=False):
    """SRJ to ||r_k|| <= tol ||r_0||, checked at k = 0 and at every cycle end (every sweep
    for M = 1).  Returns u, sweeps, relres, status ('ok' | 'noconv' | 'diverged')."""
    u = _c64(u0).copy()
    b = rhs(f, h)
    wt = axis_weights(h, u.ndim)
    c_seq = coefficients(omega_sequence, u.ndim, wt)
    M = len(c_seq)
    r02 = residual(u, b, wt)[1]
    hist = []
    if r02 == 0.0:
        return dict(u=u, sweeps=0, relres=0.0, status="ok", history=hist)
    k = 0
    while True:
        rr = float(np.sqrt(residual(u, b, wt)[1]) / np.sqrt(r02))
        if history:
            hist.append(rr)
        if not np.isfinite(rr):
            return dict(u=u, sweeps=k, relres=rr, status="diverged", history=hist)
        if rr <= tol:
            return dict(u=u, sweeps=k, relres=rr, status="ok", history=hist)
        if k + M > max_sweeps:
            return dict(u=u, sweeps=k, relres=rr, status="noconv", history=hist)
        u = run(u, b, c_seq, M, 0, wt)
        k += M


def _inner(nd):
    return tuple(slice(1, -1) for _ in range(nd))


def eigenvalues(shape_interior, wt=None):
    """lambda = sum_i a_i 4 sin^2(k_i pi / (2 N_i)), k_i = 0..N_i - 1 (array axis order; x last)."""
    nd = len(shape_interior)
    wts = (1.0, 1.0, 1.0) if wt is None else (1.0, float(wt[0]), float(wt[1]))
    lam = np.zeros(tuple(shape_interior))
    for ax, n in enumerate(shape_interior):
        k = np.arange(n, dtype=np.float64)
        g = wts[nd - 1 - ax] * 4.0 * np.sin(k * np.pi / (2.0 * n)) ** 2
        shp = [1] * nd
        shp[ax] = n
        lam = lam + g.reshape(shp)
    return lam


def dct(x):
    return scipy.fft.dctn(x, type=2, norm="ortho", workers=-1)


def predicted_relres(u0, b, omega, q, cycles, wt=None):
    """Exact-arithmetic ||r_m|| / ||r_0|| after m = 0..cycles full cycles, from the DCT-II
    modes: r^_m = b^ - lambda u^_m, u^_m = u^* + G^m (u^_0 - u^*) on every mode with
    lambda > 0 (G = prod (1 - w_i kappa)^q_i, kappa = lambda / dg); the constant mode of r is
    the mean of b and stays."""
    from .spectral import cycle_factor

    nd = np.asarray(u0).ndim
    inn = _inner(nd)
    bh = dct(np.asarray(b, dtype=np.float64)[inn])
    uh = dct(np.asarray(u0, dtype=np.float64)[inn])
    lam = eigenvalues(bh.shape, wt)
    dg = 2.0 * nd if wt is None else float(wt[2])
    nz = lam > 0
    ustar = np.zeros_like(uh)
    ustar[nz] = bh[nz] / lam[nz]
    e0 = np.where(nz, uh - ustar, 0.0)
    G = cycle_factor(omega, q, lam / dg)
    r0 = np.where(nz, -lam * e0, bh)
    out = []
    e = e0
    for m in range(cycles + 1):
        r = np.where(nz, -lam * e, bh)
        out.append(float(np.linalg.norm(r) / np.linalg.norm(r0)))
        e = G * e
    return np.array(out)


def relres_after(u0, b, omega, q, m, wt=None):
    """Exact-arithmetic ||r|| / ||r_0|| after m full cycles (any m >= 0), from the DCT-II
    modes as in predicted_relres, with G^m taken as sign and magnitude."""
    from .spectral import cycle_factor

    nd = np.asarray(u0).ndim
    inn = _inner(nd)
    bh = dct(np.asarray(b, dtype=np.float64)[inn])
    uh = dct(np.asarray(u0, dtype=np.float64)[inn])
    lam = eigenvalues(bh.shape, wt)
    dg = 2.0 * nd if wt is None else float(wt[2])
    nz = lam > 0
    ustar = np.zeros_like(uh)
    ustar[nz] = bh[nz] / lam[nz]
    e0 = np.where(nz, uh - ustar, 0.0)
    G = cycle_factor(omega, q, lam / dg)
    with np.errstate(divide="ignore", under="ignore"):
        mag = np.exp(float(m) * np.log(np.abs(G)))
    sgn = np.where((G < 0) & (int(m) % 2 == 1), -1.0, 1.0)
    r = np.where(nz, -lam * e0 * sgn * mag, bh)
    r0 = np.where(nz, -lam * e0, bh)
    return float(np.linalg.norm(r) / np.linalg.norm(r0))


def cycles_to(u0, b, omega, q, tol, wt=None, hi=1 << 40):
    """Smallest m with relres_after(m) <= tol (bisection; the relres decreases in m once the
    slowest mode dominates, which holds for the tolerances used here)."""
    lo, up = 0, 1
    while relres_after(u0, b, omega, q, up, wt) > tol:
        lo, up = up, up * 2
        if up > hi:
            raise RuntimeError("tolerance not reached")
    while up - lo > 1:
        mid = (lo + up) // 2
        if relres_after(u0, b, omega, q, mid, wt) > tol:
            lo = mid
        else:
            up = mid
    return up


def kappa_min(n_cells, h=None):
    """Smallest nonzero Jacobi symbol of the Neumann grid of n_i cells (Eq. boundaries1D3D with
    equal spacings; with h = (h_x, h_y[, h_z]) the axis weights of ``sweeps.axis_weights``)."""
    d = len(n_cells)
    wt = axis_weights(h, d) if h is not None else np.array([1.0, 1.0, 2.0 * d])
    a = (1.0, float(wt[0]), float(wt[1]))
    return min(4.0 * a[i] * np.sin(np.pi / (2.0 * n)) ** 2 for i, n in enumerate(n_cells)) / float(wt[2])
