"""Variable-coefficient operators with a mask (Sec. 5.3's Grad-Shafranov tests; Sec. 5.2's
variable-coefficient stencils) -- oracle side, test infrastructure.

The operator is given per point: (A u)_P = a_P u_P - sum over the 2d neighbours of a_nb u_nb,
with coef = [a_P, a_W, a_E, a_S, a_N (, a_D, a_U)] arrays of the full-grid shape (W/E along x,
the last array axis; S/N along y; D/U along z).  The equation is A u = f at every interior
point whose mask is 0; masked points and the ring hold fixed (Dirichlet) values, which lets the
iteration run inside a region of any shape (Sec. 5.3, test B).

Jacobi scaling, one IEEE division per coefficient: w_nb = a_nb / a_P, bs = f / a_P.  One step
with weight omega (Eq. 2nd-order_CD for this operator):
    s = (w_W W + w_E E) + (w_S S + w_N N) [+ (w_D D + w_U U)];  t = (s + bs) - u;  u' = u + omega t.
t is the Jacobi-scaled residual D^-1 (f - A u); relres = ||t||_2 / ||t_0||_2 with t_0 the scaled
residual of the state whose free points are zero (source plus fixed values), checked at k = 0
and at every cycle end.
"""
import ctypes

import numpy as np

from ._clib import lib
from .sweeps import _c64, _dims, _p


def _shape_args(u):
    d = _dims(u)
    return (d[0], d[1], d[2] if u.ndim == 3 else 1, u.ndim)


def scale(coef, f):
    """(wts, bs): the 2d neighbour weight arrays a_nb / a_P stacked, and f / a_P."""
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nnb = coef.shape[0] - 1
    n = f.size
    wts = np.empty((nnb,) + f.shape)
    bs = np.empty_like(f)
    lib().or_op_scale(n, ctypes.c_int(nnb), _p(coef), _p(wts), _p(f), _p(bs))
    return wts, bs


def _mask(mask, u):
    if mask is None:
        return None
    return np.ascontiguousarray(mask, dtype=np.uint8)


def sweep(u, wts, bs, omega, mask=None):
    u = _c64(u)
    out = u.copy()
    m = _mask(mask, u)
    nx, ny, nz, nd = _shape_args(u)
    lib().or_op_sweep(nx, ny, nz, ctypes.c_int(nd), _p(u), _p(wts), _p(bs), _p(m) if m is not None else None,
                      float(omega), _p(out))
    return out


def run(u, wts, bs, omegas, nsweeps, k0=0, mask=None):
    u = _c64(u).copy()
    M = len(omegas)
    for s in range(nsweeps):
        u = sweep(u, wts, bs, omegas[(k0 + s) % M], mask)
    return u


def residual(u, wts, bs, mask=None, zero_free=False):
    """(t field with zeros at masked points and on the ring, sum t^2, max |t|)."""
    u = _c64(u)
    m = _mask(mask, u)
    nx, ny, nz, nd = _shape_args(u)
    r = np.empty_like(u)
    out = np.zeros(2)
    rs = np.zeros(ny * nz)
    rm = np.zeros(ny * nz)
    scratch = np.empty_like(u)
    lib().or_op_residual(nx, ny, nz, ctypes.c_int(nd), _p(u), _p(wts), _p(bs), _p(m) if m is not None else None,
                         ctypes.c_int(1 if zero_free else 0), _p(r), _p(out), _p(rs), _p(rm), _p(scratch))
    return r, float(out[0]), float(out[1])


def solve(u0, f, coef, omega_sequence, tol, max_sweeps, mask=None, history=False):
    """SRJ on the operator to relres <= tol (cycle ends).  Returns u, sweeps, relres, status."""
    u = _c64(u0).copy()
    wts, bs = scale(coef, f)
    omegas = np.asarray(omega_sequence, dtype=np.float64)
    M = len(omegas)
    t02 = residual(u, wts, bs, mask, zero_free=True)[1]
    hist = []
    if t02 == 0.0:
        inner = tuple(slice(1, -1) for _ in range(u.ndim))
        free = np.ones(u.shape, bool) if mask is None else (np.asarray(mask) == 0)
        sel = np.zeros(u.shape, bool)
        sel[inner] = True
        u[sel & free] = 0.0
        return dict(u=u, sweeps=0, relres=0.0, status="ok", history=hist)
    k = 0
    while True:
        rr = float(np.sqrt(residual(u, wts, bs, mask)[1]) / np.sqrt(t02))
        if history:
            hist.append(rr)
        if not np.isfinite(rr):
            return dict(u=u, sweeps=k, relres=rr, status="diverged", history=hist)
        if rr <= tol:
            return dict(u=u, sweeps=k, relres=rr, status="ok", history=hist)
        if k + M > max_sweeps:
            return dict(u=u, sweeps=k, relres=rr, status="noconv", history=hist)
        u = run(u, wts, bs, omegas, M, 0, mask)
        k += M


def dense_system(coef, f, u_fixed, mask=None):
    """(A, rhs, free) of the equations at the free points, assembled point by point from the
    coefficients: the fixed values (ring and masked points) move to the right-hand side.
    Tiny grids only."""
    coef = np.asarray(coef, dtype=np.float64)
    shape = f.shape
    nd = len(shape)
    inner = np.zeros(shape, bool)
    inner[tuple(slice(1, -1) for _ in range(nd))] = True
    free = inner & (np.ones(shape, bool) if mask is None else (np.asarray(mask) == 0))
    idx = -np.ones(shape, dtype=np.int64)
    pts = np.argwhere(free)
    for k, p in enumerate(pts):
        idx[tuple(p)] = k
    n = len(pts)
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    # neighbour order of coef[1:]: -x, +x, -y, +y, -z, +z with x the last array axis
    offs = []
    for ax in reversed(range(nd)):
        for d in (-1, 1):
            o = [0] * nd
            o[ax] = d
            offs.append(tuple(o))
    for k, p in enumerate(pts):
        p = tuple(p)
        A[k, k] = coef[0][p]
        rhs[k] = f[p]
        for m, o in enumerate(offs):
            q = tuple(a + b for a, b in zip(p, o))
            a_nb = coef[m + 1][p]
            if idx[q] >= 0:
                A[k, idx[q]] -= a_nb
            else:
                rhs[k] += a_nb * u_fixed[q]
    return A, rhs, free


def dense_system_sparse(coef, f, u_fixed, mask=None):
    """dense_system assembled in sparse (COO) form, for grids too large for a dense matrix."""
    import scipy.sparse

    coef = np.asarray(coef, dtype=np.float64)
    shape = f.shape
    nd = len(shape)
    inner = np.zeros(shape, bool)
    inner[tuple(slice(1, -1) for _ in range(nd))] = True
    free = inner & (np.ones(shape, bool) if mask is None else (np.asarray(mask) == 0))
    idx = -np.ones(shape, dtype=np.int64)
    pts = np.argwhere(free)
    idx[tuple(pts.T)] = np.arange(len(pts))
    rows, cols, vals = [np.arange(len(pts))], [np.arange(len(pts))], [coef[0][tuple(pts.T)]]
    rhs = np.array(f[tuple(pts.T)], dtype=np.float64)
    m = 0
    for ax in reversed(range(nd)):
        for d in (-1, 1):
            q = pts.copy()
            q[:, ax] += d
            a_nb = coef[m + 1][tuple(pts.T)]
            qi = idx[tuple(q.T)]
            inside = qi >= 0
            rows.append(np.nonzero(inside)[0])
            cols.append(qi[inside])
            vals.append(-a_nb[inside])
            rhs[~inside] += a_nb[~inside] * np.asarray(u_fixed)[tuple(q[~inside].T)]
            m += 1
    A = scipy.sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(len(pts), len(pts)))
    return A, rhs, free
