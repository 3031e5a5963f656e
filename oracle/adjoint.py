"""Dense-solve gradients of L = 1/2 ||u - u_target||^2 -- oracle side (test infrastructure).

The discrete problem is A u = b~ with A = 2d I - (interior neighbour couplings) (units
of h^2, symmetric) and b~_P = h^2 f_P + sum of the ring values g_e adjacent to P (the
Poisson form of Sec. 5.1 with Dirichlet data).  For the quadratic loss
    lambda = A^-1 (u - u_target),   dL/df_P = h^2 lambda_P,   dL/dg_e = lambda_{P(e)},
where P(e) is the interior cell next to ring cell e.  Ring cells that no stencil reads
(corners in 2D; edges and corners in 3D) get zero.  With unequal spacings (h a tuple) the
equation is multiplied through by h_x^2: dL/df_P = h_x^2 lambda_P and dL/dg_e = a(e)
lambda_{P(e)}, a(e) the weight of the axis along which P(e) reads e.
"""
import numpy as np

from . import spectral


def _inner(nd):
    return tuple(slice(1, -1) for _ in range(nd))


def _weights(h, nd):
    from .sweeps import axis_weights

    return None if np.isscalar(h) else axis_weights(h, nd)


def _hx(h):
    return float(h) if np.isscalar(h) else float(h[0])


def forward_dense(f, g_ring, h):
    """u on the full grid (ring = g_ring) from the dense LU solve."""
    b = np.zeros_like(np.asarray(f, dtype=np.float64))
    nd = b.ndim
    b[_inner(nd)] = (_hx(h) * _hx(h)) * np.asarray(f, dtype=np.float64)[_inner(nd)]
    return spectral.dense_solve(g_ring, b, _weights(h, nd))


def loss(u, u_target):
    nd = u.ndim
    d = (u - u_target)[_inner(nd)]
    return 0.5 * float(np.sum(d * d))


def grad_dense(f, g_ring, u_target, h):
    """(dL/df, dL/dg) as full-grid arrays: dL/df zero on the ring, dL/dg zero inside."""
    u = forward_dense(f, g_ring, h)
    nd = u.ndim
    wt = _weights(h, nd)
    rhs = np.zeros_like(u)
    rhs[_inner(nd)] = (u - u_target)[_inner(nd)]
    lam = spectral.dense_solve(np.zeros_like(u), rhs, wt)  # A lambda = u - u_t, zero ring
    df = np.zeros_like(u)
    df[_inner(nd)] = (_hx(h) * _hx(h)) * lam[_inner(nd)]
    dg = np.zeros_like(u)
    for ax in range(nd):
        for side, src in ((0, 1), (-1, -2)):
            dst_idx = [slice(1, -1)] * nd
            src_idx = [slice(1, -1)] * nd
            dst_idx[ax] = side
            src_idx[ax] = src
            dg[tuple(dst_idx)] = spectral.axis_weight(wt, nd, ax) * lam[tuple(src_idx)]
    return df, dg
