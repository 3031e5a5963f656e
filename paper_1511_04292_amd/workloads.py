"""Seeded synthetic inputs for the SRJ solver (host numpy, FP64).

This module only draws and shapes input data; it holds none of the solver's arithmetic
and is shared by the tests, the benchmark and the smoke check.  Every array has the
full-grid shape with its Dirichlet ring: (n_y + 2, n_x + 2) in 2D, (n_z + 2, n_y + 2,
n_x + 2) in 3D, x fastest, spacing h = 1 / (n + 1) on the unit square / cube.

Random streams are numpy ``default_rng`` (PCG64) with the seeds given per workload.
"""
import math

import numpy as np


def grid_spacing(n):
    return 1.0 / (n + 1)


def coords(n):
    return np.arange(n + 2, dtype=np.float64) * grid_spacing(n)


def _set_ring_zero(a):
    a[0, ...] = 0.0
    a[-1, ...] = 0.0
    if a.ndim >= 2:
        a[:, 0, ...] = 0.0
        a[:, -1, ...] = 0.0
    if a.ndim == 3:
        a[:, :, 0] = 0.0
        a[:, :, -1] = 0.0
    return a


def random_ring(shape_full, rng, lo=-1.0, hi=1.0):
    """Array of the full-grid shape: U(lo, hi) on the ring, 0 inside (corners included)."""
    g = rng.uniform(lo, hi, size=shape_full)
    inner = tuple(slice(1, -1) for _ in shape_full)
    g[inner] = 0.0
    return g


def gaussian_blobs_2d(n, count, rng, sigma=(0.01, 0.1)):
    """sum_j a_j exp(-((x-cx_j)^2 + (y-cy_j)^2) / (2 s_j^2)); centres U(0,1)^2,
    s_j ~ U(sigma), a_j ~ N(0, 1); zero on the ring."""
    x = coords(n)
    cx = rng.uniform(0.0, 1.0, count)
    cy = rng.uniform(0.0, 1.0, count)
    s = rng.uniform(sigma[0], sigma[1], count)
    a = rng.standard_normal(count)
    f = np.zeros((n + 2, n + 2))
    for j in range(count):
        gx = np.exp(-((x - cx[j]) ** 2) / (2.0 * s[j] ** 2))
        gy = np.exp(-((x - cy[j]) ** 2) / (2.0 * s[j] ** 2))
        f += a[j] * np.outer(gy, gx)
    return _set_ring_zero(f)


def manufactured_noise_2d(n, seed=0, noise=1e-3):
    """f = 2 pi^2 sin(pi x) sin(pi y) + N(0, noise^2) per interior point; ring 0."""
    rng = np.random.default_rng(seed)
    x = coords(n)
    f = 2.0 * math.pi ** 2 * np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
    f[1:-1, 1:-1] += rng.normal(0.0, noise, size=(n, n))
    return _set_ring_zero(f)


def six_neighbour_mean(v):
    """(1/6) sum of the six axis neighbours, with zero outside the interior (input shaping
    for the 3D workload)."""
    p = np.zeros_like(v)
    p[1:-1, 1:-1, 1:-1] = v[1:-1, 1:-1, 1:-1]
    out = np.zeros_like(v)
    out[1:-1, 1:-1, 1:-1] = (p[1:-1, 1:-1, :-2] + p[1:-1, 1:-1, 2:] + p[1:-1, :-2, 1:-1] +
                             p[1:-1, 2:, 1:-1] + p[:-2, 1:-1, 1:-1] + p[2:, 1:-1, 1:-1]) / 6.0
    return out


# ------------------------------------------------------------------ workloads

def small_2d(n=64, seed=0):
    """64 x 64 interior, zero ring, f = manufactured sin-sin source + N(0, 1e-3^2) noise."""
    f = manufactured_noise_2d(n, seed)
    u0 = np.zeros_like(f)
    return dict(n=(n, n), h=grid_spacing(n), u0=u0, f=f)


def blobs_2d(n=4096, seed=0, count=32):
    """n x n interior, ring U(-1,1), f = 32 Gaussian blobs; u0 interior zero."""
    rng = np.random.default_rng(seed)
    u0 = random_ring((n + 2, n + 2), rng)
    f = gaussian_blobs_2d(n, count, rng)
    return dict(n=(n, n), h=grid_spacing(n), u0=u0, f=f)


def smooth_3d(n=512, seed=0):
    """n^3 interior, zero ring, f = U(-1,1) i.i.d. then one six-neighbour mean."""
    rng = np.random.default_rng(seed)
    v = np.zeros((n + 2, n + 2, n + 2))
    v[1:-1, 1:-1, 1:-1] = rng.uniform(-1.0, 1.0, size=(n, n, n))
    f = six_neighbour_mean(v)
    u0 = np.zeros_like(f)
    return dict(n=(n, n, n), h=grid_spacing(n), u0=u0, f=f)


def batch_sizes(count=1024, seed=3, lo=32, hi=1024, plo=3, phi=8):
    """Side N_j = floor(exp(U(ln lo, ln hi))) and levels P_j ~ U{plo..phi}.  Sides are not
    powers of two: a draw that lands on one moves to the next integer (to the previous one
    at the upper end of the range)."""
    rng = np.random.default_rng(seed)
    N = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)
    N = np.clip(N, lo, hi)
    pow2 = (N & (N - 1)) == 0
    N = np.where(pow2, np.where(N + 1 <= hi, N + 1, N - 1), N)
    P = rng.integers(plo, phi + 1, size=count)
    return N, P


def batch_problem(n, seed):
    """One batch member: f ~ N(0,1) i.i.d. inside, zero ring, zero start."""
    rng = np.random.default_rng(seed)
    f = np.zeros((n + 2, n + 2))
    f[1:-1, 1:-1] = rng.standard_normal((n, n))
    return dict(n=(n, n), h=grid_spacing(n), u0=np.zeros_like(f), f=f)


def adjoint_2d(n=2048, seed=0, target_seed=1):
    """f = Gaussian blobs, boundary U(-1,1), u_target a blob field from another seed."""
    rng = np.random.default_rng(seed)
    g = random_ring((n + 2, n + 2), rng)
    f = gaussian_blobs_2d(n, 32, rng)
    rt = np.random.default_rng(target_seed)
    ut = gaussian_blobs_2d(n, 32, rt)
    return dict(n=(n, n), h=grid_spacing(n), g=g, f=f, u_target=ut)


def random_state(shape_full, seed):
    """Random field with a random ring (for single-sweep parity checks)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=shape_full)


def blobs_2d_device(n, seed=0, count=32, device="cuda:0"):
    """A blob workload too large to draw on the host quickly (e.g. 32768^2, 8.6 GB per array):
    ring U(-1,1) drawn edge by edge (top row, bottom row, left column, right column, corners
    included), then 32 blobs as in gaussian_blobs_2d, all from one PCG64 stream; the arrays
    are assembled on the device in binary64 (torch).  The same distribution as blobs_2d, not
    the same values."""
    import torch

    rng = np.random.default_rng(seed)
    m = n + 2
    top, bottom = rng.uniform(-1.0, 1.0, m), rng.uniform(-1.0, 1.0, m)
    left, right = rng.uniform(-1.0, 1.0, n), rng.uniform(-1.0, 1.0, n)
    cx = rng.uniform(0.0, 1.0, count)
    cy = rng.uniform(0.0, 1.0, count)
    s = rng.uniform(0.01, 0.1, count)
    a = rng.standard_normal(count)
    dt = torch.float64
    u0 = torch.zeros((m, m), dtype=dt, device=device)
    u0[0, :] = torch.from_numpy(top).to(device)
    u0[-1, :] = torch.from_numpy(bottom).to(device)
    u0[1:-1, 0] = torch.from_numpy(left).to(device)
    u0[1:-1, -1] = torch.from_numpy(right).to(device)
    x = torch.from_numpy(coords(n)).to(device)
    f = torch.zeros((m, m), dtype=dt, device=device)
    for j in range(count):
        gx = torch.exp(-((x - float(cx[j])) ** 2) / (2.0 * float(s[j]) ** 2))
        gy = torch.exp(-((x - float(cy[j])) ** 2) / (2.0 * float(s[j]) ** 2))
        f.add_(torch.outer(gy, gx), alpha=float(a[j]))
    f[0, :] = 0.0
    f[-1, :] = 0.0
    f[:, 0] = 0.0
    f[:, -1] = 0.0
    return dict(n=(n, n), h=grid_spacing(n), u0=u0, f=f)


def exp_xy_unit_square(nx_zones=585, ny_zones=280):
    """The Dirichlet test problem of Sec. 5.1 on the unit square cut into nx_zones x ny_zones
    uniform zones: interior points (nx_zones - 1) x (ny_zones - 1), spacings
    h = (1/nx_zones, 1/ny_zones).  With -lap(u) = f the source is f = (x^2 + y^2) e^(xy) and
    the ring holds the exact solution u = -e^(xy) (so u(0, y) = u(x, 0) = -1, u(1, y) = -e^y,
    u(x, 1) = -e^x).  Returns n, h, u0 (ring set, interior 0), f (ring 0) and u_exact on the
    full grid."""
    nx, ny = nx_zones - 1, ny_zones - 1
    hx, hy = 1.0 / nx_zones, 1.0 / ny_zones
    x = np.arange(nx + 2, dtype=np.float64) * hx
    y = np.arange(ny + 2, dtype=np.float64) * hy
    X, Y = np.meshgrid(x, y, indexing="xy")
    ue = -np.exp(X * Y)
    f = (X * X + Y * Y) * np.exp(X * Y)
    f[0, :] = f[-1, :] = 0.0
    f[:, 0] = f[:, -1] = 0.0
    u0 = ue.copy()
    u0[1:-1, 1:-1] = 0.0
    return dict(n=(nx, ny), h=(hx, hy), u0=u0, f=f, u_exact=ue)


def grad_shafranov(n=298, C=0.0, test="A"):
    """The linear Grad-Shafranov problem of Sec. 5.3, Delta* Psi + C^2 Psi = 0 with
    Delta* = d_rr + r^-2 d_thth - cot(th) r^-2 d_th, on r in [1, 10], th in [0, pi], with
    n x n interior points (n + 2 equispaced points per axis including the boundaries: the
    paper's 300 x 300 grid is n = 298).  x (the fastest axis) is r, y is theta.

    Written as A Psi = 0 with A = -(Delta* + C^2) discretised by second-order central
    differences: a_W = a_E = 1/h_r^2, a_S = 1/(r^2 h_th^2) + cot(th)/(2 r^2 h_th),
    a_N = 1/(r^2 h_th^2) - cot(th)/(2 r^2 h_th), a_P = 2/h_r^2 + 2/(r^2 h_th^2) - C^2.
    Test A: Psi = sin^2(th)/r at r = 1 and r = 10, 0 at th = 0, pi (exact solution for C = 0:
    sin^2(th)/r).  Test B: the same operator solved only inside the region r < R(th) of
    Eq. shape_b with the disk (r sin th - 4)^2 + (r cos th - 1.6)^2 < 1 removed; Psi = 0 outside
    it (a mask) and on the outer boundaries, Psi = sin^2(pi (th - th1)/(th2 - th1)) on r = 1 for
    th1 = 0.3037 <= th <= th2 = 2.8903.  The start is 0 everywhere inside.
    Returns n, coef (5, n+2, n+2), u0, f (zeros), mask (uint8 or None), r, theta and, for test
    A, u_exact."""
    m = n + 2
    r = 1.0 + 9.0 * np.arange(m, dtype=np.float64) / (m - 1)
    th = math.pi * np.arange(m, dtype=np.float64) / (m - 1)
    hr, ht = 9.0 / (m - 1), math.pi / (m - 1)
    R, TH = np.meshgrid(r, th, indexing="xy")
    coef = np.zeros((5, m, m))
    with np.errstate(divide="ignore", invalid="ignore"):
        cot = np.cos(TH) / np.sin(TH)
    inv_r2 = 1.0 / (R * R)
    coef[0] = 2.0 / (hr * hr) + 2.0 * inv_r2 / (ht * ht) - C * C
    coef[1] = 1.0 / (hr * hr)
    coef[2] = 1.0 / (hr * hr)
    coef[3] = inv_r2 / (ht * ht) + cot * inv_r2 / (2.0 * ht)
    coef[4] = inv_r2 / (ht * ht) - cot * inv_r2 / (2.0 * ht)
    ring = np.ones((m, m), bool)
    ring[1:-1, 1:-1] = False
    coef[:, ring] = 0.0
    coef[0, ring] = 1.0
    u0 = np.zeros((m, m))
    out = dict(n=(n, n), coef=coef, f=np.zeros((m, m)), r=r, theta=th, mask=None)
    if test == "A":
        u0[:, 0] = np.sin(th) ** 2 / r[0]
        u0[:, -1] = np.sin(th) ** 2 / r[-1]
        u0[0, :] = u0[-1, :] = 0.0
        out["u_exact"] = np.sin(TH) ** 2 / R
    else:
        shape = (4.5 * np.sin(TH) ** 2 + 2.5 * np.sin(2 * TH) ** 2) * (
            1 - 0.4 * np.cos(3 * TH) + 0.3 * np.cos(5 * TH) + 0.05 * np.sin(25 * TH))
        disk = (R * np.sin(TH) - 4.0) ** 2 + (R * np.cos(TH) - 1.6) ** 2 < 1.0
        inside = (R < shape) & ~disk
        th1, th2 = 0.3037, 2.8903
        on = (th >= th1) & (th <= th2)
        u0[:, 0] = np.where(on, np.sin((th - th1) / (th2 - th1) * math.pi) ** 2, 0.0)
        mask = np.zeros((m, m), np.uint8)
        mask[1:-1, 1:-1] = (~inside[1:-1, 1:-1]).astype(np.uint8)
        out["mask"] = mask
    out["u0"] = u0
    return out


def _sph_first_zero(l):
    """First positive zero of the spherical Bessel function j_l (bracketed scan, then brentq)."""
    from scipy.optimize import brentq
    from scipy.special import spherical_jn

    x = max(1.0, float(l))
    step = 0.05
    f0 = spherical_jn(l, x)
    while True:
        x1 = x + step
        f1 = spherical_jn(l, x1)
        if f0 == 0.0:
            return x
        if f0 * f1 < 0.0:
            return brentq(lambda t: spherical_jn(l, t), x, x1, xtol=1e-15, rtol=1e-15, maxiter=200)
        x, f0 = x1, f1


def spherical_series(r, theta, terms=30):
    """Sec. 5.2's axisymmetric test (m_max = 0, n_max -> infinity): the source
    s = -sum_n a_2n k_2n^2 j_2n(k_2n r) Y_2n^0(theta) for r <= 1 (0 outside) and the solution
    u = sum_n (a_2n j_2n(k_2n r) + b_2n r^2n) Y_2n^0 for r <= 1, sum_n b_2n r^-(2n+1) Y_2n^0 for
    r > 1, with a_l = 2^-l, k_l the first zero of j_l, b_l = -a_l/(2l+1) (l j_l(k_l) - k_l
    j_(l+1)(k_l)) and Y_l^0 = sqrt((2l+1)/(4 pi)) P_l(cos theta).  The terms fall as 4^-n: the
    sum stops at 30 terms, far below binary64 resolution.  Returns (s, u) on the broadcast of
    r and theta."""
    from scipy.special import eval_legendre, spherical_jn

    r = np.asarray(r, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    s = np.zeros(np.broadcast(r, theta).shape)
    u = np.zeros_like(s)
    inside = r <= 1.0
    for nn in range(terms):
        l = 2 * nn
        a = 2.0 ** (-l)
        k = _sph_first_zero(l)
        b = -a / (2 * l + 1) * (l * spherical_jn(l, k) - k * spherical_jn(l + 1, k))
        Y = math.sqrt((2 * l + 1) / (4.0 * math.pi)) * eval_legendre(l, np.cos(theta))
        jr = spherical_jn(l, k * np.where(inside, r, 1.0))
        s = s + np.where(inside, -a * k * k * jr, 0.0) * Y
        u = u + np.where(inside, a * jr + b * r ** l, b * np.where(inside, 1.0, r) ** (-(l + 1))) * Y
    return s, u


def spherical_poisson_2d(N, start="zero", seed=0):
    """Sec. 5.2's Poisson equation in spherical coordinates, axisymmetric (r, theta) on
    [0, 1] x [0, pi] with N x N cells, multiplied by r^2 and discretised by second-order central
    differences on the staggered grid r_i = (i - 1/2)/N, theta_j = (j - 1/2) pi / N
    (x, the fastest axis, is r; y is theta):
        r^2 (u_E - 2u + u_W)/dr^2 + r (u_E - u_W)/dr + (u_N - 2u + u_S)/dth^2
        + cot(theta) (u_N - u_S)/(2 dth) = r^2 s,
    written as A u = f with A = -(that operator), f = -r^2 s: a_W = r (r - dr)/dr^2,
    a_E = r (r + dr)/dr^2, a_S = 1/dth^2 - cot/(2 dth), a_N = 1/dth^2 + cot/(2 dth),
    a_P = 2 r^2/dr^2 + 2/dth^2.  Boundaries: at the centre u_0 = u_1 = u_2, so the unknowns in
    r are i = 2..N and the first one's diagonal takes a_W in (a_P - a_W, a_W = 0); at theta = 0
    and pi a ghost cell mirrors its neighbour (a_P - a_S resp. a_P - a_N); at r_(N+1) =
    1 + dr/2 the ring holds the exact exterior solution.  Interior: (N - 1) x N points.
    start: "zero" (the paper's ab initio calculation) or "realistic": the exact solution times
    (1 + U(-1/2, 1/2)/N) per point, seeded.  Returns n, coef (5, N+2, N+1), u0, f, r, theta,
    u_exact (on the full grid) and h (dr, dth)."""
    dr, dth = 1.0 / N, math.pi / N
    ri = (np.arange(1, N + 2) - 0.5) * dr          # x = 0 .. N  <->  i = 1 .. N+1
    tj = (np.arange(0, N + 2) - 0.5) * dth         # y = 0 .. N+1 <->  j = 0 .. N+1
    R, TH = np.meshgrid(ri, tj, indexing="xy")
    my, mx = N + 2, N + 1
    with np.errstate(divide="ignore", invalid="ignore"):
        cot = np.cos(TH) / np.sin(TH)
    coef = np.zeros((5, my, mx))
    coef[1] = R * (R - dr) / (dr * dr)
    coef[2] = R * (R + dr) / (dr * dr)
    coef[3] = 1.0 / (dth * dth) - cot / (2.0 * dth)
    coef[4] = 1.0 / (dth * dth) + cot / (2.0 * dth)
    coef[0] = 2.0 * R * R / (dr * dr) + 2.0 / (dth * dth)
    # folds: centre (x = 1 is i = 2: u_1 = u_2), axis ghosts at theta = 0 (y = 1) and pi (y = N)
    coef[0, :, 1] -= coef[1, :, 1]
    coef[1, :, 1] = 0.0
    coef[0, 1, :] -= coef[3, 1, :]
    coef[3, 1, :] = 0.0
    coef[0, N, :] -= coef[4, N, :]
    coef[4, N, :] = 0.0
    ring = np.ones((my, mx), bool)
    ring[1:-1, 1:-1] = False
    coef[:, ring] = 0.0
    coef[0, ring] = 1.0
    s_src, u_ex = spherical_series(R, TH)
    f = np.where(ring, 0.0, -(R * R) * s_src)
    u0 = np.zeros((my, mx))
    u0[1:-1, -1] = u_ex[1:-1, -1]  # r_(N+1) = 1 + dr/2: the exterior solution
    if start == "realistic":
        rng = np.random.default_rng(seed)
        u0[1:-1, 1:-1] = u_ex[1:-1, 1:-1] * (1.0 + rng.uniform(-0.5, 0.5, (N, N - 1)) / N)
    elif start != "zero":
        raise ValueError("start is 'zero' or 'realistic'")
    return dict(n=(N - 1, N), coef=coef, u0=u0, f=f, r=ri, theta=tj, u_exact=u_ex, h=(dr, dth))
