"""Weighted-Jacobi sweeps, SRJ cycles, residuals and the stopping rule -- oracle side.

Test infrastructure only (see ``oracle/__init__``).  Arrays are numpy, C-contiguous,
shape ``(n_y + 2, n_x + 2)`` in 2D or ``(n_z + 2, n_y + 2, n_x + 2)`` in 3D; index 0 and
``n + 1`` of each axis is the Dirichlet ring.  Axis ``-1`` (x) is the fastest.

Paper passages followed:
* one step omega_i J -- Sec. 3.1, Eq. 2nd-order_CD (Poisson form, -lap u = f, b = h^2 f);
  on a box whose axes have different spacings (the unit square of Sec. 5.1 cut into
  585 x 280 zones) the equation is multiplied through by h_x^2: weight 1 on the x
  neighbours, wy = h_x^2 / h_y^2 and wz = h_x^2 / h_z^2 on the others, diagonal
  dg = 2 ((1 + wy) + wz), b = h_x^2 f and c = omega / dg (``axis_weights``);
* the M-cycle, weight i applied q_i times, cycles repeated -- Sec. 2;
* the residual used to stop: r = b - A u with A = 2d I - (sum of neighbours) in units
  of h^2; relres = ||r||_2 / ||b~||_2 with b~ the residual of the zero interior (source
  plus boundary terms).  The paper's own stopping figure ||u^n - u^(n-1)||_inf
  (Sec. 4.1, footnote on the tolerance) is reported beside it.
"""
import ctypes

import numpy as np

from ._clib import lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(u):
    if u.ndim == 2:
        return (u.shape[1] - 2, u.shape[0] - 2)
    if u.ndim == 3:
        return (u.shape[2] - 2, u.shape[1] - 2, u.shape[0] - 2)
    raise ValueError("2D or 3D arrays only")


def _c64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _hx(h):
    return float(h) if np.isscalar(h) else float(h[0])


def axis_weights(h, ndim):
    """wt = (wy, wz, dg) for spacing h: a number (every axis) or (h_x, h_y[, h_z]).
    wy = h_x^2 / h_y^2, wz = h_x^2 / h_z^2 (1 in 2D), dg = 2 (1 + wy) in 2D and
    2 ((1 + wy) + wz) in 3D; equal spacings give (1, 1, 2d) exactly."""
    hs = (float(h),) * ndim if np.isscalar(h) else tuple(float(x) for x in h)
    if len(hs) != ndim:
        raise ValueError("one spacing per axis")
    hxx = hs[0] * hs[0]
    wy = hxx / (hs[1] * hs[1])
    wz = hxx / (hs[2] * hs[2]) if ndim == 3 else 1.0
    dg = 2.0 * (1.0 + wy) if ndim == 2 else 2.0 * ((1.0 + wy) + wz)
    return np.array([wy, wz, dg], dtype=np.float64)


def _wt(wt, ndim):
    if wt is None:
        return np.array([1.0, 1.0, 2.0 * ndim], dtype=np.float64)
    return np.ascontiguousarray(wt, dtype=np.float64)


def rhs(f, h):
    """b = (h_x*h_x) * f on the interior, 0 on the ring (h_x*h_x is rounded once, then the
    product); h is the spacing of every axis or (h_x, h_y[, h_z])."""
    f = _c64(f)
    hh = _hx(h) * _hx(h)
    b = np.zeros_like(f)
    inner = tuple(slice(1, -1) for _ in range(f.ndim))
    b[inner] = hh * f[inner]
    return b


def sweep(u, b, c, wt=None):
    """One weighted-Jacobi step with coefficient c = omega / dg  (Eq. 2nd-order_CD); wt the
    axis weights (default: equal spacings)."""
    u = _c64(u)
    b = _c64(b)
    w = _wt(wt, u.ndim)
    out = u.copy()
    L = lib()
    d = _dims(u)
    if u.ndim == 2:
        L.or_sweep2d(d[0], d[1], _p(u), _p(b), _p(w), float(c), _p(out))
    else:
        L.or_sweep3d(d[0], d[1], d[2], _p(u), _p(b), _p(w), float(c), _p(out))
    return out


def jacobi(u, b):
    """One plain Jacobi step from its own definition, u' = (sum of neighbours + b) / (2d)
    (equal spacings)."""
    u = _c64(u)
    b = _c64(b)
    out = u.copy()
    L = lib()
    d = _dims(u)
    if u.ndim == 2:
        L.or_jacobi2d(d[0], d[1], _p(u), _p(b), _p(out))
    else:
        L.or_jacobi3d(d[0], d[1], d[2], _p(u), _p(b), _p(out))
    return out


def coefficients(omega_sequence, ndim, wt=None):
    """c_k = omega_k / dg for an ordered weight sequence (one IEEE division each; dg = 2d for
    equal spacings)."""
    w = np.asarray(omega_sequence, dtype=np.float64)
    return w / float(_wt(wt, ndim)[2])


def run(u, b, c_seq, nsweeps, k0=0, wt=None):
    """Apply ``nsweeps`` scheduled steps; step s uses c_seq[(k0 + s) mod M] (Sec. 2)."""
    u = _c64(u).copy()
    b = _c64(b)
    w = _wt(wt, u.ndim)
    c_seq = np.ascontiguousarray(c_seq, dtype=np.float64)
    work = u.copy()
    L = lib()
    d = _dims(u)
    if u.ndim == 2:
        L.or_srj2d(d[0], d[1], _p(u), _p(b), _p(w), _p(c_seq), len(c_seq), int(k0), int(nsweeps), _p(work))
    else:
        L.or_srj3d(d[0], d[1], d[2], _p(u), _p(b), _p(w), _p(c_seq), len(c_seq), int(k0), int(nsweeps),
                   _p(work))
    return u


def residual_norms(u, b, wt=None):
    """(sum r^2, max |r|) of r = b - A u on the interior, compensated summation."""
    u = _c64(u)
    b = _c64(b)
    w = _wt(wt, u.ndim)
    L = lib()
    d = _dims(u)
    out = np.zeros(2)
    if u.ndim == 2:
        rs = np.zeros(d[1])
        rm = np.zeros(d[1])
        L.or_residual2d(d[0], d[1], _p(u), _p(b), _p(w), _p(out), _p(rs), _p(rm))
    else:
        rs = np.zeros(d[1] * d[2])
        rm = np.zeros(d[1] * d[2])
        L.or_residual3d(d[0], d[1], d[2], _p(u), _p(b), _p(w), _p(out), _p(rs), _p(rm))
    return float(out[0]), float(out[1])


def residual_field(u, b, wt=None):
    """r = b - A u on the interior, 0 on the ring."""
    u = _c64(u)
    b = _c64(b)
    w = _wt(wt, u.ndim)
    r = np.empty_like(u)
    L = lib()
    d = _dims(u)
    if u.ndim == 2:
        L.or_residual_field2d(d[0], d[1], _p(u), _p(b), _p(w), _p(r))
    else:
        L.or_residual_field3d(d[0], d[1], d[2], _p(u), _p(b), _p(w), _p(r))
    return r


def zero_interior(u):
    z = np.array(u, dtype=np.float64, copy=True)
    z[tuple(slice(1, -1) for _ in range(z.ndim))] = 0.0
    return z


def source_norm2(u, b, wt=None):
    """||b~||_2^2: the squared residual of the state whose interior is zero."""
    return residual_norms(zero_interior(u), b, wt)[0]


def relres(u, b, bt2=None, wt=None):
    if bt2 is None:
        bt2 = source_norm2(u, b, wt)
    r2, _ = residual_norms(u, b, wt)
    return float(np.sqrt(r2) / np.sqrt(bt2)) if bt2 > 0 else 0.0


def solve(u0, f, h, omega_sequence, tol, max_sweeps, history=False):
    """SRJ to a relative residual: checks at k = 0 and at every cycle end (k = 0 mod M).

    h is the spacing of every axis or one per axis (h_x, h_y[, h_z]).  Returns a dict with
    u, sweeps, relres, status ('ok' | 'noconv' | 'diverged') and, if ``history``, the relres
    at every check.  Plain Jacobi is the one-weight schedule [1.0] and is then checked after
    every sweep.
    """
    u = _c64(u0).copy()
    b = rhs(f, h)
    wt = axis_weights(h, u.ndim)
    c_seq = coefficients(omega_sequence, u.ndim, wt)
    M = len(c_seq)
    bt2 = source_norm2(u, b, wt)
    hist = []
    if bt2 == 0.0:
        # zero source and zero boundary: u = 0 is exact
        u[tuple(slice(1, -1) for _ in range(u.ndim))] = 0.0
        return dict(u=u, sweeps=0, relres=0.0, status="ok", history=hist)
    k = 0
    while True:
        r2, _ = residual_norms(u, b, wt)
        rr = float(np.sqrt(r2) / np.sqrt(bt2))
        if history:
            hist.append(rr)
        if not np.isfinite(rr):
            return dict(u=u, sweeps=k, relres=rr, status="diverged", history=hist)
        if rr <= tol:
            return dict(u=u, sweeps=k, relres=rr, status="ok", history=hist)
        if k + M > max_sweeps:
            return dict(u=u, sweeps=k, relres=rr, status="noconv", history=hist)
        u = run(u, b, c_seq, M, k0=0, wt=wt)
        k += M


# ----------------------------------------------------------- reduced precision

def to_bf16_bits(x32):
    """binary32 -> bfloat16 bit patterns, round to nearest, ties to even."""
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    out = np.empty(x32.shape, dtype=np.uint16)
    lib().or_f32_to_bf16(x32.size, _p(x32), _p(out))
    return out


def from_bf16_bits(h):
    h = np.ascontiguousarray(h, dtype=np.uint16)
    out = np.empty(h.shape, dtype=np.float32)
    lib().or_bf16_to_f32(h.size, _p(h), _p(out))
    return out


def sweep_lo(u, b, c32, fmt, wt=None):
    """One step in binary32 arithmetic; storage binary32 ('f32') or bfloat16 bits ('bf16'),
    with the binary32 roundings of the axis weights.  'f64' is the binary64 step itself
    (refinement with binary64 inner sweeps)."""
    if fmt == "f64":
        return sweep(u, b, c32, wt)
    w32 = _wt(wt, u.ndim).astype(np.float32)
    L = lib()
    d = _dims(u)
    out = u.copy()
    if fmt == "f32":
        if u.ndim == 2:
            L.or_sweep2d_f32(d[0], d[1], _p(u), _p(b), _p(w32), float(c32), _p(out))
        else:
            L.or_sweep3d_f32(d[0], d[1], d[2], _p(u), _p(b), _p(w32), float(c32), _p(out))
    elif fmt == "bf16":
        if u.ndim == 2:
            L.or_sweep2d_bf16(d[0], d[1], _p(u), _p(b), _p(w32), float(c32), _p(out))
        else:
            L.or_sweep3d_bf16(d[0], d[1], d[2], _p(u), _p(b), _p(w32), float(c32), _p(out))
    else:
        raise ValueError(fmt)
    return out


def lo_coefficients(omega_sequence, ndim, fmt="f32", wt=None):
    """Coefficients of the sweep format: the FP64 c_k, rounded once to binary32 unless the
    format is 'f64'."""
    c = coefficients(omega_sequence, ndim, wt)
    return c if fmt == "f64" else c.astype(np.float32)


def lo_cast(x64, fmt):
    """FP64 -> storage format: binary32 rounding, then (bf16) a second rounding to bfloat16;
    'f64' is a copy."""
    if fmt == "f64":
        return np.array(x64, dtype=np.float64, copy=True)
    x32 = np.ascontiguousarray(x64, dtype=np.float32)
    return x32 if fmt == "f32" else to_bf16_bits(x32)


def lo_widen(x, fmt):
    return (x if fmt in ("f32", "f64") else from_bf16_bits(x)).astype(np.float64)


def solve_ir(u0, f, h, omega_sequence, tol, inner_cycles, max_outer, fmt):
    """FP64 iterative refinement around low-precision SRJ sweeps.

    Outer step: r = b - A u in FP64; stop if ||r|| / ||b~|| <= tol; otherwise solve
    A d = r approximately by ``inner_cycles`` SRJ cycles from d = 0 with a zero ring,
    in binary32 arithmetic on ``fmt`` storage (r cast to that storage first), then
    u += d in FP64.  ``fmt`` 'f64' runs the same loop with binary64 inner sweeps.
    Pinned by: with one binary64 cycle per outer step it is the plain iteration (same stop,
    iterates equal to rounding); with binary32 each outer step contracts ||r|| by the exact
    cycle factor's maximum (Eq. cycleAmplFact) up to rounding; both storage formats end within
    the conditioning bound of the exact discrete solution.
    """
    u = _c64(u0).copy()
    b = rhs(f, h)
    wt = axis_weights(h, u.ndim)
    c32 = lo_coefficients(omega_sequence, u.ndim, fmt, wt)
    M = len(c32)
    bt2 = source_norm2(u, b, wt)
    inner = tuple(slice(1, -1) for _ in range(u.ndim))
    hist = []
    sweeps = 0
    for outer in range(max_outer + 1):
        r = residual_field(u, b, wt)
        rr = float(np.sqrt(residual_norms(u, b, wt)[0]) / np.sqrt(bt2)) if bt2 > 0 else 0.0
        hist.append(rr)
        if not np.isfinite(rr):
            return dict(u=u, outer=outer, sweeps=sweeps, relres=rr, status="diverged", history=hist)
        if rr <= tol:
            return dict(u=u, outer=outer, sweeps=sweeps, relres=rr, status="ok", history=hist)
        if outer == max_outer:
            break
        rl = lo_cast(r, fmt)
        d = lo_cast(np.zeros_like(u), fmt)
        for s in range(inner_cycles * M):
            d = sweep_lo(d, rl, c32[s % M], fmt, wt)
        sweeps += inner_cycles * M
        u[inner] = u[inner] + lo_widen(d, fmt)[inner]
    return dict(u=u, outer=max_outer, sweeps=sweeps, relres=hist[-1], status="noconv", history=hist)
