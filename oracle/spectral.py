"""Exact solutions and closed forms that pin the oracle's sweeps -- test infrastructure.

The Dirichlet 5-/7-point Laplacian on a box of n_i interior points per axis (spacing h)
is diagonalised by the separable type-I discrete sine transform: the mode
(k_1..k_d), k_i = 1..n_i, has eigenvalue lambda = sum_i 4 sin^2(k_i pi / (2 (n_i+1)))
of A = 2d I - (sum of neighbours).  Its Jacobi symbol is kappa = lambda / (2d), which
is the paper's kappa of Sec. 3.1 (Eq. boundaries, Eq. boundaries1D3D), written for
Dirichlet boundaries with N_i = n_i + 1 zones (Eq. effectiveNDirichlet).

With unequal spacings (axis weights wt = (wy, wz, dg) of ``sweeps.axis_weights``) the same
transform diagonalises A = dg I - (weighted neighbour sum): lambda = sum_i a_i 4 sin^2(..),
a_i the weight of axis i (1 for x), and kappa = lambda / dg.  Arrays are indexed (z,) y, x,
so array axis nd - 1 carries weight 1, nd - 2 weight wy and nd - 3 weight wz.

A weighted-Jacobi step with weight w multiplies the error in every mode by
G_w(kappa) = 1 - w kappa (Sec. 3.1); a full M-cycle multiplies it by
prod_i (1 - w_i kappa)^q_i (Eq. cycleAmplFact), whatever the order of the steps.
"""
import numpy as np
import scipy.fft
import scipy.linalg


def _inner(ndim):
    return tuple(slice(1, -1) for _ in range(ndim))


def axis_weight(wt, nd, ax):
    """Weight of array axis ax of an nd-dimensional array (x last): 1, wy, wz."""
    if wt is None:
        return 1.0
    return (1.0, float(wt[0]), float(wt[1]))[nd - 1 - ax]


def diagonal(wt, nd):
    return 2.0 * nd if wt is None else float(wt[2])


def load_vector(u_ring, b, wt=None):
    """b~ = b + (weighted boundary neighbour sums): the right-hand side of A u = b~ on the
    interior."""
    u_ring = np.asarray(u_ring, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nd = u_ring.ndim
    g = np.array(u_ring, copy=True)
    g[_inner(nd)] = 0.0
    acc = np.array(b[_inner(nd)], copy=True)
    for ax in range(nd):
        lo = [slice(1, -1)] * nd
        hi = [slice(1, -1)] * nd
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        acc += axis_weight(wt, nd, ax) * (g[tuple(lo)] + g[tuple(hi)])
    return acc


def eigenvalues(shape_interior, wt=None):
    """lambda over all modes, array of the interior shape (axis order as the arrays)."""
    nd = len(shape_interior)
    grids = []
    for ax, n in enumerate(shape_interior):
        k = np.arange(1, n + 1, dtype=np.float64)
        grids.append(axis_weight(wt, nd, ax) * (4.0 * np.sin(k * np.pi / (2.0 * (n + 1))) ** 2))
    lam = np.zeros(tuple(shape_interior))
    for ax, g in enumerate(grids):
        shp = [1] * nd
        shp[ax] = len(g)
        lam = lam + g.reshape(shp)
    return lam


def kappas(shape_interior, wt=None):
    """Jacobi symbols kappa = lambda / dg (dg = 2d with equal spacings) of every mode."""
    return eigenvalues(shape_interior, wt) / diagonal(wt, len(shape_interior))


def dst(x):
    """Orthonormal type-I DST over every axis (its own inverse); the per-axis transforms run
    on all host threads."""
    return scipy.fft.dstn(x, type=1, norm="ortho", workers=-1)


def exact_solve(u_ring, b, wt=None):
    """u* = A^-1 b~ by the DST-I diagonalisation; ring copied from u_ring."""
    rhs = load_vector(u_ring, b, wt)
    lam = eigenvalues(rhs.shape, wt)
    u = np.array(u_ring, dtype=np.float64, copy=True)
    u[_inner(u.ndim)] = dst(dst(rhs) / lam)
    return u


def dense_matrix(shape_interior, wt=None):
    """A = dg I - (weighted interior neighbour couplings), assembled explicitly (tiny grids
    only); dg = 2d and unit weights with equal spacings."""
    shape = tuple(shape_interior)
    n = int(np.prod(shape))
    d = len(shape)
    A = np.zeros((n, n))
    idx = np.arange(n).reshape(shape)
    A[np.arange(n), np.arange(n)] = diagonal(wt, d)
    for ax in range(d):
        a = [slice(None)] * d
        c = [slice(None)] * d
        a[ax] = slice(0, -1)
        c[ax] = slice(1, None)
        i0 = idx[tuple(a)].ravel()
        i1 = idx[tuple(c)].ravel()
        A[i0, i1] = -axis_weight(wt, d, ax)
        A[i1, i0] = -axis_weight(wt, d, ax)
    return A


def dense_solve(u_ring, b, wt=None):
    """u* from an LU factorisation of the assembled matrix (tiny grids)."""
    rhs = load_vector(u_ring, b, wt)
    A = dense_matrix(rhs.shape, wt)
    x = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), rhs.ravel())
    u = np.array(u_ring, dtype=np.float64, copy=True)
    u[_inner(u.ndim)] = x.reshape(rhs.shape)
    return u


def manufactured_2d(n):
    """Discrete solution for f = 2 pi^2 sin(pi x) sin(pi y), zero ring, h = 1/(n+1).

    sin(pi x) sin(pi y) is the (1,1) eigenvector, so u_h = (t / sin t)^2 sin sin with
    t = pi h / 2.  Returns (x, y, u_h, f) on the full grid with its ring.
    """
    h = 1.0 / (n + 1)
    x = np.arange(n + 2) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    s = np.sin(np.pi * X) * np.sin(np.pi * Y)
    t = np.pi * h / 2.0
    u = (t / np.sin(t)) ** 2 * s
    f = 2.0 * np.pi ** 2 * s
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
    f[0, :] = f[-1, :] = f[:, 0] = f[:, -1] = 0.0
    return x, x, u, f


def cycle_factor(omega, q, kappa):
    """prod_i (1 - w_i kappa)^q_i  (Eq. cycleAmplFact), elementwise over kappa.

    The factors are accumulated as a sign and a sum of q_i log|1 - w_i kappa|: single powers
    such as (1 - w kappa)^q overflow binary64 for the large weights and counts of P >= 8
    schemes although the full product is small."""
    kappa = np.asarray(kappa, dtype=np.float64)
    logmag = np.zeros_like(kappa)
    sign = np.ones_like(kappa)
    with np.errstate(divide="ignore"):
        for w, qi in zip(omega, q):
            base = 1.0 - float(w) * kappa
            logmag = logmag + int(qi) * np.log(np.abs(base))
            if int(qi) % 2 == 1:
                sign = sign * np.sign(base)
    return sign * np.exp(logmag)


def cycle_amplification(omega, q, shape_interior, wt=None):
    """max over the discrete spectrum of |prod_i (1 - w_i kappa)^q_i|."""
    return float(np.max(np.abs(cycle_factor(omega, q, kappas(shape_interior, wt)))))


def predicted_relres(u0, b, omega, q, cycles, wt=None):
    """Exact-arithmetic relres after m full cycles, m = 0..cycles, from the DST modes.

    e_m = G^m e_0 mode by mode, r = -A e, relres_m = ||lambda G^m e_0|| / ||b~||.
    """
    rhs = load_vector(u0, b, wt)
    lam = eigenvalues(rhs.shape, wt)
    ustar = dst(dst(rhs) / lam)
    e0 = dst(np.asarray(u0, dtype=np.float64)[_inner(rhs.ndim)] - ustar)
    G = cycle_factor(omega, q, lam / diagonal(wt, rhs.ndim))
    bn = np.linalg.norm(rhs)
    out = []
    e = e0
    for m in range(cycles + 1):
        out.append(float(np.linalg.norm(lam * e) / bn))
        e = G * e
    return np.array(out)


def predicted_state(u0, b, omega, q, cycles, wt=None):
    """Exact-arithmetic iterate after ``cycles`` full M-cycles (interior from DST modes)."""
    rhs = load_vector(u0, b, wt)
    lam = eigenvalues(rhs.shape, wt)
    ustar_hat = dst(rhs) / lam
    e0 = dst(np.asarray(u0, dtype=np.float64)[_inner(rhs.ndim)]) - ustar_hat
    G = cycle_factor(omega, q, lam / diagonal(wt, rhs.ndim))
    u = np.array(u0, dtype=np.float64, copy=True)
    u[_inner(u.ndim)] = dst(ustar_hat + G ** cycles * e0)
    return u
