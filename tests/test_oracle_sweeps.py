"""Pins of the oracle's sweeps, residuals and stopping rule against closed forms, library
routines and brute force (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import schedule, spectral, sweeps
from paper_1511_04292_amd import workloads


def _rand_problem(shape_interior, seed):
    rng = np.random.default_rng(seed)
    full = tuple(n + 2 for n in shape_interior)
    u = workloads.random_ring(full, rng)
    f = np.zeros(full)
    f[tuple(slice(1, -1) for _ in full)] = rng.standard_normal(tuple(shape_interior))
    return u, f


@pytest.mark.parametrize("shape", [(9, 12), (4, 6, 5)])
def test_dst_solve_equals_dense_lu(shape):
    u, f = _rand_problem(shape, 1)
    b = sweeps.rhs(f, 0.1)
    a = spectral.exact_solve(u, b)
    d = spectral.dense_solve(u, b)
    assert np.max(np.abs(a - d)) <= 1e-12 * np.max(np.abs(d))


@pytest.mark.parametrize("shape", [(17, 23), (6, 7, 5)])
def test_residual_of_exact_solution_vanishes(shape):
    u, f = _rand_problem(shape, 2)
    b = sweeps.rhs(f, 1.0 / 24)
    us = spectral.exact_solve(u, b)
    r2, rmax = sweeps.residual_norms(us, b)
    scale = np.max(np.abs(spectral.load_vector(u, b)))
    assert rmax <= 1e-12 * scale
    # and the source norm is the norm of the load vector b~ (ring terms included)
    assert math.isclose(sweeps.source_norm2(u, b), float(np.sum(spectral.load_vector(u, b) ** 2)),
                        rel_tol=1e-13)


def test_residual_sum_is_exactly_rounded_sum():
    u, f = _rand_problem((40, 33), 3)
    u[1:-1, 1:-1] = np.random.default_rng(4).standard_normal((40, 33)) * 1e3
    b = sweeps.rhs(f, 0.3)
    r = sweeps.residual_field(u, b)
    r2, rmax = sweeps.residual_norms(u, b)
    exact = math.fsum(float(x) * float(x) for x in r[1:-1, 1:-1].ravel())
    assert abs(r2 - exact) <= 4e-16 * exact
    assert rmax == float(np.max(np.abs(r)))


@pytest.mark.parametrize("shape", [(11, 8), (5, 4, 6)])
def test_single_sweep_matches_matrix_form(shape):
    # u' = u + c (b~ - A u) with A assembled as a dense matrix (independent route)
    rng = np.random.default_rng(5)
    full = tuple(n + 2 for n in shape)
    u = rng.uniform(-1, 1, size=full)
    f = rng.uniform(-1, 1, size=full)
    b = sweeps.rhs(f, 0.05)
    c = 37.5 / (2 * len(shape))
    out = sweeps.sweep(u, b, c)
    A = spectral.dense_matrix(shape)
    inner = tuple(slice(1, -1) for _ in shape)
    x = u[inner].ravel()
    ref = x + c * (spectral.load_vector(u, b).ravel() - A @ x)
    scale = np.max(np.abs(u)) * (1 + 2 * len(shape) * abs(c)) + abs(c) * np.max(np.abs(b))
    assert np.max(np.abs(out[inner].ravel() - ref)) <= 8e-16 * scale
    # ring untouched
    ring = np.ones(full, bool)
    ring[inner] = False
    assert np.array_equal(out[ring], u[ring])


@pytest.mark.parametrize("ndim", [2, 3])
def test_unit_weight_reduces_to_jacobi(ndim):
    shape = (20, 17) if ndim == 2 else (9, 8, 7)
    u, f = _rand_problem(shape, 6)
    b = sweeps.rhs(f, 0.05)
    a = sweeps.run(u, b, sweeps.coefficients([1.0], ndim), 1000)
    j = u.copy()
    for _ in range(1000):
        j = sweeps.jacobi(j, b)
    assert np.max(np.abs(a - j)) <= 1e-13 * np.max(np.abs(j))


def test_cycles_follow_exact_modal_trajectory():
    # after m full cycles the iterate is G^m e_0 + u* in every DST mode (Eq. cycleAmplFact)
    shape = (23, 31)
    u, f = _rand_problem(shape, 7)
    b = sweeps.rhs(f, 1.0 / 32)
    omega = [120.0, 9.0, 0.8]
    q = [1, 4, 20]
    seq = [0] + [2] * 5 + [1] + [2] * 5 + [1, 2, 2, 2, 2, 1] + [2] * 5 + [1] + [2]
    assert sorted(seq) == sorted(sum(([i] * qi for i, qi in enumerate(q)), []))
    wseq = np.array(omega)[seq]
    M = len(seq)
    for m in (1, 2, 5):
        got = sweeps.run(u, b, sweeps.coefficients(wseq, 2), m * M)
        ref = spectral.predicted_state(u, b, omega, q, m)
        assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_cycle_amplification_equals_spectral_radius():
    # brute force: the one-cycle iteration matrix on a tiny grid, its eigenvalues
    shape = (4, 3)
    omega = [9.5, 0.7]
    q = [1, 3]
    seq = [1, 0, 1, 1]
    A = spectral.dense_matrix(shape)
    n = A.shape[0]
    E = np.eye(n)
    for i in seq:
        E = (np.eye(n) - (omega[i] / 4.0) * A) @ E
    rad = float(np.max(np.abs(np.linalg.eigvals(E))))
    assert math.isclose(spectral.cycle_amplification(omega, q, shape), rad, rel_tol=1e-10)


def test_jacobi_relres_matches_prediction():
    shape = (15, 15)
    u, f = _rand_problem(shape, 8)
    b = sweeps.rhs(f, 1.0 / 16)
    res = sweeps.solve(u, f, 1.0 / 16, [1.0], 1e-30, 60, history=True)
    pred = spectral.predicted_relres(u, b, [1.0], [1], 60)
    np.testing.assert_allclose(res["history"], pred, rtol=1e-9)


def test_manufactured_solution_closed_form():
    n = 64
    x, y, uh, f = spectral.manufactured_2d(n)
    b = sweeps.rhs(f, 1.0 / (n + 1))
    us = spectral.exact_solve(np.zeros_like(f), b)
    assert np.max(np.abs(us - uh)) <= 1e-13
    t = math.pi / (2 * (n + 1))
    X, Y = np.meshgrid(x, y, indexing="xy")
    s = np.sin(math.pi * X) * np.sin(math.pi * Y)
    err = np.max(np.abs(uh - s))
    assert math.isclose(err, ((t / math.sin(t)) ** 2 - 1.0) * np.max(s), rel_tol=1e-9)
    assert 1.94e-4 < err < 1.95e-4  # about pi^2 h^2 / 12


def test_solve_stops_at_first_cycle_end_below_tol():
    w = workloads.small_2d(24, seed=1)
    opt = schedule.optimal(2, schedule.kappa_min_dirichlet([24, 24]))
    q = schedule.q_floor(opt["beta"])
    seq = schedule.weight_sequence(opt["w"], schedule.order_even(q))
    res = sweeps.solve(w["u0"], w["f"], w["h"], seq, 1e-6, 10 ** 6, history=True)
    hist = res["history"]
    assert res["status"] == "ok"
    assert hist[-1] <= 1e-6 and all(hh > 1e-6 for hh in hist[:-1])
    assert res["sweeps"] == len(seq) * (len(hist) - 1)
    us = spectral.exact_solve(w["u0"], sweeps.rhs(w["f"], w["h"]))
    cond = 8.0 / (8.0 * math.sin(math.pi / 50) ** 2)
    assert np.max(np.abs(res["u"] - us)) <= 2 * cond * 1e-6 * np.max(np.abs(us))


def test_zero_source_and_boundary_returns_immediately():
    u = np.zeros((10, 10))
    u[3, 3] = 5.0
    res = sweeps.solve(u, np.zeros((10, 10)), 0.1, [1.0], 1e-10, 100)
    assert res["sweeps"] == 0 and res["status"] == "ok" and not np.any(res["u"])


def test_noconv_when_budget_too_small():
    w = workloads.small_2d(16, seed=2)
    res = sweeps.solve(w["u0"], w["f"], w["h"], [1.0], 1e-10, 10)
    assert res["status"] == "noconv" and res["sweeps"] == 10


def test_nan_source_reports_divergence():
    w = workloads.small_2d(16, seed=2)
    w["f"][5, 5] = np.nan
    res = sweeps.solve(w["u0"], w["f"], w["h"], [1.0], 1e-10, 10)
    assert res["status"] == "diverged"


def test_f32_sweep_within_binary32_rounding():
    rng = np.random.default_rng(9)
    u = rng.uniform(-1, 1, size=(30, 41))
    b = rng.uniform(-1e-3, 1e-3, size=(30, 41))
    c64 = 1234.5 / 4.0
    out64 = sweeps.sweep(u.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64),
                         float(np.float32(c64)))
    out32 = sweeps.sweep_lo(u.astype(np.float32), b.astype(np.float32), np.float32(c64), "f32")
    bound = 8 * 2.0 ** -24 * (np.abs(u) * (1 + 4 * c64) + 4 * c64 * 1.0 + c64 * 1e-3)
    assert np.all(np.abs(out32.astype(np.float64) - out64) <= bound + 1e-30)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(10)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.0e38, -0.0,
                                  np.inf, -np.inf, 1e-40, 2 ** -126], dtype=np.float32)])
    mine = sweeps.to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(mine, ref)
    back = sweeps.from_bf16_bits(mine)
    assert np.array_equal(back, torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16).float().numpy())


def test_ir_reaches_tolerance_in_both_formats():
    w = workloads.small_2d(31, seed=3)
    km = schedule.kappa_min_dirichlet([31, 31])
    opt = schedule.optimal(3, km)
    q = schedule.q_floor(opt["beta"])
    seq = schedule.weight_sequence(opt["w"], schedule.order_balanced(opt["w"], q, km))
    us = spectral.exact_solve(w["u0"], sweeps.rhs(w["f"], w["h"]))
    for fmt in ("f32", "bf16"):
        res = sweeps.solve_ir(w["u0"], w["f"], w["h"], seq, 1e-10, 4, 60, fmt)
        assert res["status"] == "ok", (fmt, res["history"][-5:])
        assert np.max(np.abs(res["u"] - us)) <= 1e-7 * np.max(np.abs(us))


def _ir_case(n, P):
    w = workloads.small_2d(n, seed=3)
    km = schedule.kappa_min_dirichlet([n, n])
    opt = schedule.optimal(P, km)
    q = schedule.q_floor(opt["beta"])
    seq = schedule.weight_sequence(opt["w"], schedule.order_balanced(opt["w"], q, km))
    return w, opt, q, seq


@pytest.mark.parametrize("n,P", [(31, 3), (40, 5)])
def test_ir_f64_one_cycle_is_the_plain_iteration(n, P):
    """Refinement with one binary64 cycle per outer step is, in exact arithmetic, the plain
    SRJ iteration cycle by cycle (the error goes e -> G e either way, G the cycle's
    propagation matrix of Sec. 2): same stopping cycle, iterates equal to rounding."""
    w, opt, q, seq = _ir_case(n, P)
    M = len(seq)
    ref = sweeps.solve(w["u0"], w["f"], w["h"], seq, 1e-10, 10 ** 6, history=True)
    ir = sweeps.solve_ir(w["u0"], w["f"], w["h"], seq, 1e-10, 1, 10 ** 4, "f64")
    assert ref["status"] == ir["status"] == "ok"
    assert ir["outer"] == ref["sweeps"] // M and ir["sweeps"] == ref["sweeps"]
    assert np.max(np.abs(ir["u"] - ref["u"])) <= 1e-13 * np.max(np.abs(ref["u"]))
    hr, hi = np.array(ref["history"]), np.array(ir["history"])
    big = hr > 1e-7  # above the residual's rounding floor
    np.testing.assert_allclose(hi[big], hr[big], rtol=1e-6)


@pytest.mark.parametrize("n,P", [(31, 3), (40, 5)])
def test_ir_f32_outer_steps_contract_by_the_cycle_factor(n, P):
    """Each outer step with one binary32 cycle reduces ||r||_2 by at most the cycle's exact
    contraction max over the grid's symbols of |prod (1 - w_i kappa)^q_i| (Eq.
    cycleAmplFact; the cycle operator is symmetric, so this is its 2-norm), up to binary32
    rounding (slack 1e-3)."""
    w, opt, q, seq = _ir_case(n, P)
    gmax = spectral.cycle_amplification(opt["w"], q, (n, n))
    r = sweeps.solve_ir(w["u0"], w["f"], w["h"], seq, 1e-10, 1, 10 ** 4, "f32")
    assert r["status"] == "ok"
    h = np.array(r["history"])
    assert np.all(h[1:] <= (gmax + 1e-3) * h[:-1]), (gmax, (h[1:] / h[:-1]).max())


def test_modal_prediction_with_large_schedule():
    # P = 10 scheme: single powers (1 - w kappa)^q overflow, the cycle factor must not;
    # two full cycles of the oracle's sweeps follow the exact modal relres
    n = (95, 95)
    wl = workloads.blobs_2d(95, seed=3)
    km = schedule.kappa_min_dirichlet(n)
    o = schedule.optimal(10, km)
    q = schedule.q_floor(o["beta"])
    G = spectral.cycle_factor(o["w"], q, spectral.kappas(n))
    assert np.all(np.isfinite(G)) and np.max(np.abs(G)) < 1.0
    seq = schedule.order_balanced(o["w"], q, km)
    b = sweeps.rhs(wl["f"], wl["h"])
    M = int(np.sum(q))
    u = sweeps.run(wl["u0"], b, sweeps.coefficients(np.asarray(o["w"])[seq], 2), 2 * M)
    pred = spectral.predicted_relres(wl["u0"], b, o["w"], q, 2)
    got = sweeps.relres(u, b)
    assert abs(got - pred[2]) <= 1e-3 * pred[2]


def _matrix_form_step(x_full, b_full, c):
    """u + c (b~ - A u) on the interior from the dense matrix (independent route), FP64."""
    shape = tuple(n - 2 for n in x_full.shape)
    inner = tuple(slice(1, -1) for _ in shape)
    A = spectral.dense_matrix(shape)
    x = x_full[inner].ravel()
    return (x + c * (spectral.load_vector(x_full, b_full).ravel() - A @ x)).reshape(shape)


def _step_bound(x_full, b_full, c):
    """Per-point bound on the rounding of one binary32 step: 8 units of 2^-24 times the
    magnitudes entering it (|u| + |c| (sum |neighbours| + |b| + 2d |u|))."""
    nd = x_full.ndim
    inner = tuple(slice(1, -1) for _ in range(nd))
    a = np.abs(x_full)
    nb = np.zeros(tuple(n - 2 for n in x_full.shape))
    for ax in range(nd):
        lo = [slice(1, -1)] * nd
        hi = [slice(1, -1)] * nd
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        nb += a[tuple(lo)] + a[tuple(hi)]
    return 8 * 2.0 ** -24 * (a[inner] + abs(c) * (nb + np.abs(b_full[inner]) + 2 * nd * a[inner]))


@pytest.mark.parametrize("fmt,shape", [("f32", (5, 4, 6)), ("bf16", (13, 9)), ("bf16", (5, 6, 4)),
                                       ("f32", (9, 14))])
def test_lo_sweep_matches_matrix_form(fmt, shape):
    """The binary32 and bfloat16-storage steps against the dense matrix form evaluated in
    FP64 from the same stored inputs: binary32 results within the per-term rounding bound;
    bfloat16 results equal to the bfloat16 rounding of a value within that bound."""
    rng = np.random.default_rng(11)
    full = tuple(n + 2 for n in shape)
    nd = len(shape)
    u = rng.uniform(-1, 1, size=full)
    b = rng.uniform(-1e-3, 1e-3, size=full)
    c32 = np.float32(1234.5 / (2 * nd))
    c = float(c32)
    inner = tuple(slice(1, -1) for _ in shape)
    if fmt == "f32":
        u_s, b_s = u.astype(np.float32), b.astype(np.float32)
        x, bx = u_s.astype(np.float64), b_s.astype(np.float64)
    else:
        u_s, b_s = sweeps.to_bf16_bits(u.astype(np.float32)), sweeps.to_bf16_bits(b.astype(np.float32))
        x, bx = sweeps.from_bf16_bits(u_s).astype(np.float64), sweeps.from_bf16_bits(b_s).astype(np.float64)
    out = sweeps.sweep_lo(u_s, b_s, c32, fmt)
    got = out.astype(np.float64) if fmt == "f32" else sweeps.from_bf16_bits(out).astype(np.float64)
    ref = _matrix_form_step(x, bx, c)
    bound = _step_bound(x, bx, c)
    if fmt == "f32":
        assert np.all(np.abs(got[inner] - ref) <= bound)
    else:
        lo = sweeps.from_bf16_bits(sweeps.to_bf16_bits((ref - bound).astype(np.float32))).astype(np.float64)
        hi = sweeps.from_bf16_bits(sweeps.to_bf16_bits((ref + bound).astype(np.float32))).astype(np.float64)
        assert np.all((lo <= got[inner]) & (got[inner] <= hi))
    ring = np.ones(full, bool)
    ring[inner] = False
    assert np.array_equal(out[ring], u_s[ring])


# ------------------------------------------------------- unequal spacings (Sec. 5.1 case)

H2 = (1.0 / 12, 1.0 / 7)         # h_x, h_y
H3 = (1.0 / 6, 1.0 / 9, 1.0 / 4)  # h_x, h_y, h_z


def _weighted_dense_by_hand(shape_interior_xyz, h):
    """-lap_h * h_x^2 assembled from its definition, one coupling at a time (independent of
    spectral.dense_matrix): off-diagonals -(h_x/h_i)^2 on axis i, diagonal their sum twice."""
    nd = len(shape_interior_xyz)
    n = int(np.prod(shape_interior_xyz))
    A = np.zeros((n, n))

    def idx(p):  # p = (x, y[, z]) -> row-major index with x fastest
        k = 0
        for a in reversed(range(nd)):
            k = k * shape_interior_xyz[a] + p[a]
        return k

    for flat in range(n):
        p, r = [], flat
        for a in range(nd):
            p.append(r % shape_interior_xyz[a])
            r //= shape_interior_xyz[a]
        for a in range(nd):
            wa = (h[0] / h[a]) ** 2
            A[flat, flat] += 2 * wa
            for d in (-1, 1):
                q = list(p)
                q[a] += d
                if 0 <= q[a] < shape_interior_xyz[a]:
                    A[flat, idx(q)] -= wa
    return A


@pytest.mark.parametrize("h", [H2, H3])
def test_weighted_matrix_and_weights(h):
    nd = len(h)
    shape_xyz = (5, 4) if nd == 2 else (3, 4, 2)
    wt = sweeps.axis_weights(h, nd)
    A = spectral.dense_matrix(tuple(reversed(shape_xyz)), wt)
    np.testing.assert_allclose(A, _weighted_dense_by_hand(shape_xyz, h), rtol=1e-14, atol=1e-14)
    # equal spacings give unit weights and the diagonal 2d exactly
    assert list(sweeps.axis_weights(0.125, nd)) == [1.0, 1.0, 2.0 * nd]


@pytest.mark.parametrize("h", [H2, H3])
def test_weighted_sweep_matches_matrix_form(h):
    nd = len(h)
    shape = (6, 11) if nd == 2 else (5, 4, 6)  # array order (z,) y, x
    rng = np.random.default_rng(21)
    full = tuple(n + 2 for n in shape)
    u = rng.uniform(-1, 1, size=full)
    f = rng.uniform(-1, 1, size=full)
    wt = sweeps.axis_weights(h, nd)
    b = sweeps.rhs(f, h)
    c = 37.5 / wt[2]
    out = sweeps.sweep(u, b, c, wt)
    inner = tuple(slice(1, -1) for _ in shape)
    x = u[inner].ravel()
    ref = x + c * (spectral.load_vector(u, b, wt).ravel() - spectral.dense_matrix(shape, wt) @ x)
    scale = np.max(np.abs(u)) * (1 + 2 * wt[2] * abs(c)) + abs(c) * np.max(np.abs(b))
    assert np.max(np.abs(out[inner].ravel() - ref)) <= 8e-16 * scale
    # the residual loops agree with the matrix form
    r = sweeps.residual_field(u, b, wt)
    rr = spectral.load_vector(u, b, wt).ravel() - spectral.dense_matrix(shape, wt) @ x
    assert np.max(np.abs(r[inner].ravel() - rr)) <= 8e-16 * scale / abs(c)
    r2, rmax = sweeps.residual_norms(u, b, wt)
    assert math.isclose(r2, float(np.sum(rr * rr)), rel_tol=1e-13)
    assert math.isclose(rmax, float(np.max(np.abs(rr))), rel_tol=1e-13)


@pytest.mark.parametrize("h", [H2, H3])
def test_weighted_dst_solve_equals_dense_lu_and_kappa_min(h):
    nd = len(h)
    shape = (9, 12) if nd == 2 else (4, 6, 5)
    u, f = _rand_problem(shape, 22)
    wt = sweeps.axis_weights(h, nd)
    b = sweeps.rhs(f, h)
    a = spectral.exact_solve(u, b, wt)
    d = spectral.dense_solve(u, b, wt)
    assert np.max(np.abs(a - d)) <= 1e-12 * np.max(np.abs(d))
    ev = np.linalg.eigvalsh(spectral.dense_matrix(shape, wt))
    np.testing.assert_allclose(np.sort(spectral.eigenvalues(shape, wt).ravel()), ev, rtol=1e-12, atol=1e-12)
    n_xyz = tuple(reversed(shape))
    assert math.isclose(schedule.kappa_min_dirichlet(n_xyz, h), ev[0] / wt[2], rel_tol=1e-12)


def test_weighted_cycles_follow_exact_modal_trajectory():
    shape = (13, 19)
    u, f = _rand_problem(shape, 23)
    wt = sweeps.axis_weights(H2, 2)
    b = sweeps.rhs(f, H2)
    omega = [60.0, 6.0, 0.8]
    q = [1, 3, 12]
    seq = [0, 2, 2, 2, 1, 2, 2, 2, 2, 1, 2, 2, 2, 2, 1, 2]
    c = sweeps.coefficients(np.array(omega)[seq], 2, wt)
    for m in (1, 3):
        got = sweeps.run(u, b, c, m * len(seq), wt=wt)
        ref = spectral.predicted_state(u, b, omega, q, m, wt)
        assert np.max(np.abs(got - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_case_study_discretisation_is_second_order():
    """Sec. 5.1: -lap u = (x^2 + y^2) e^(xy) on the unit square with u = -e^(xy) on the
    boundary.  The exact discrete solution on 585 x 280 zones differs from -e^(xy) by
    O(h_x^2 + h_y^2): at most (h_x^2 + h_y^2) e / 96 (truncation error at most
    (h_x^2 + h_y^2) e / 12, discrete Laplacian inverse at most 1/8 in the max norm on the unit
    square), and halving both spacings divides the error by 4."""
    errs = []
    for zones in ((146, 70), (292, 140), (585, 280)):
        wl = workloads.exp_xy_unit_square(*zones)
        wt = sweeps.axis_weights(wl["h"], 2)
        us = spectral.exact_solve(wl["u0"], sweeps.rhs(wl["f"], wl["h"]), wt)
        err = float(np.max(np.abs(us - wl["u_exact"])))
        hx, hy = wl["h"]
        assert err <= (hx * hx + hy * hy) * math.e / 96
        errs.append(err)
    assert 3.95 < errs[0] / errs[1] < 4.05


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_weighted_lo_sweep_matches_matrix_form(fmt):
    rng = np.random.default_rng(24)
    shape = (7, 10)
    full = tuple(n + 2 for n in shape)
    u = rng.uniform(-1, 1, size=full)
    b = rng.uniform(-1e-3, 1e-3, size=full)
    wt = sweeps.axis_weights(H2, 2)
    w32 = wt.astype(np.float32).astype(np.float64)
    c32 = np.float32(1234.5 / wt[2])
    c = float(c32)
    inner = (slice(1, -1), slice(1, -1))
    if fmt == "f32":
        u_s, b_s = u.astype(np.float32), b.astype(np.float32)
        x, bx = u_s.astype(np.float64), b_s.astype(np.float64)
    else:
        u_s, b_s = sweeps.to_bf16_bits(u.astype(np.float32)), sweeps.to_bf16_bits(b.astype(np.float32))
        x, bx = sweeps.from_bf16_bits(u_s).astype(np.float64), sweeps.from_bf16_bits(b_s).astype(np.float64)
    out = sweeps.sweep_lo(u_s, b_s, c32, fmt, wt)
    got = out.astype(np.float64) if fmt == "f32" else sweeps.from_bf16_bits(out).astype(np.float64)
    A = spectral.dense_matrix(shape, w32)
    ref = (x[inner].ravel() + c * (spectral.load_vector(x, bx, w32).ravel() - A @ x[inner].ravel())).reshape(shape)
    a = np.abs(x)
    nb = (a[1:-1, :-2] + a[1:-1, 2:]) + w32[0] * (a[:-2, 1:-1] + a[2:, 1:-1])
    bound = 8 * 2.0 ** -24 * (a[inner] + abs(c) * (nb + np.abs(bx[inner]) + w32[2] * a[inner]))
    if fmt == "f32":
        assert np.all(np.abs(got[inner] - ref) <= bound)
    else:
        lo = sweeps.from_bf16_bits(sweeps.to_bf16_bits((ref - bound).astype(np.float32))).astype(np.float64)
        hi = sweeps.from_bf16_bits(sweeps.to_bf16_bits((ref + bound).astype(np.float32))).astype(np.float64)
        assert np.all((lo <= got[inner]) & (got[inner] <= hi))
