"""Parity at the benchmark's full sizes, in the launch configuration bench.py times.

4096^2 (P = 10), 2048^2 (P = 9) and 512^3 (P = 8) in binary64, and the binary32 and
bfloat16-storage sweeps at 4096^2 and 512^3: windows of sweeps at the default fusion depth
(10 in 2D, 4 in binary64 3D, 5 in the 4- and 2-byte formats in 3D), crossing a cycle end, are
compared bit for bit with the oracle run on the whole grid -- on the oracle's schedules and
on the schedules the product planner builds for the benchmark.  The full 4096^2 and 512^3
binary64 solves must stop at the cycle the exact DST-mode trajectory predicts, with the
relres it predicts; the 512^3 results of all three precisions are compared with the exact
discrete solution.  At 32768^2 (the throughput point) sampled regions of a window are
compared with the oracle run on crops around them.  Windows at 4800 x 4700 and 3500 x 3400
cover the fused 2D binary64 kernel in both store forms at every depth.
"""
import numpy as np
import pytest
import torch

from oracle import schedule as S
from oracle import spectral, sweeps
from paper_1511_04292_amd import srj, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

_CACHE = {}


def oracle_schedule(P, n):
    key = (P, n)
    if key not in _CACHE:
        km = S.kappa_min_dirichlet(n)
        o = S.optimal(P, km)
        q = S.q_floor(o["beta"])
        _CACHE[key] = (o["w"], q, S.order_balanced(o["w"], q, km))
    return _CACHE[key]


@pytest.fixture(scope="module")
def blobs():
    return workloads.blobs_2d(4096, seed=0)


def test_blobs_4096_window_bitwise(blobs):
    wl = blobs
    w, q, seq = oracle_schedule(10, wl["n"])
    M = int(np.sum(q))
    plan = srj.srj_plan(wl["n"], wl["h"], omega=w, q=q, sequence=seq)
    assert srj.srj_plan_describe(plan)["fused_sweeps"] == 10
    c = sweeps.coefficients(np.asarray(w)[seq], 2)
    b = sweeps.rhs(wl["f"], wl["h"])
    for k0, n in ((0, 64), (M - 21, 43)):  # the second window crosses the cycle end
        u = torch.from_numpy(wl["u0"]).to(DEV)
        srj.srj_sweeps(plan, u, torch.from_numpy(wl["f"]).to(DEV), k0, n)
        ref = sweeps.run(wl["u0"], b, c, n, k0=k0)
        assert np.array_equal(u.cpu().numpy(), ref), (k0, n)


@pytest.mark.parametrize("n,hint", [((4800, 4700), 0), ((3500, 3400), 1)])
def test_store_variants_every_depth_bitwise(n, hint):
    """The fused binary64 2D kernel in both store forms, at every depth 1..10, against the
    oracle: 23 sweeps from 7 before a cycle end.  4800 x 4700 (input, output and b beyond twice
    the memory-side cache) stores plainly, 3500 x 3400 (between once and twice) with the
    non-temporal hint."""
    h = 1.0 / (n[0] + 1)
    rng = np.random.default_rng(21)
    full = (n[1] + 2, n[0] + 2)
    u0 = rng.uniform(-1.0, 1.0, full)
    f = rng.standard_normal(full)
    w, q, seq = oracle_schedule(4, n)
    M = int(np.sum(q))
    plan = srj.srj_plan(n, h, omega=w, q=q, sequence=seq)
    assert srj.srj_plan_describe(plan)["store_nt"] == hint
    k0, nsw = M - 7, 23
    ref = sweeps.run(u0, sweeps.rhs(f, h), sweeps.coefficients(np.asarray(w)[seq], 2), nsw, k0=k0)
    fd = torch.from_numpy(f).to(DEV)
    for T in range(1, 11):
        srj.srj_plan_set_fusion(plan, T)
        u = torch.from_numpy(u0).to(DEV)
        srj.srj_sweeps(plan, u, fd, k0, nsw)
        assert np.array_equal(u.cpu().numpy(), ref), T


def test_blobs_4096_solve_stops_where_predicted(blobs):
    wl = blobs
    w, q, seq = oracle_schedule(10, wl["n"])
    M = int(np.sum(q))
    tol = 1e-10
    b = sweeps.rhs(wl["f"], wl["h"])
    pred = spectral.predicted_relres(wl["u0"], b, w, q, 12)
    m_pred = int(np.argmax(pred <= tol))
    assert pred[m_pred] <= tol
    plan = srj.srj_plan(wl["n"], wl["h"], omega=w, q=q, sequence=seq)
    u = torch.from_numpy(wl["u0"]).to(DEV)
    info = srj.srj_solve(plan, u, torch.from_numpy(wl["f"]).to(DEV), tol, 30 * M)
    assert info["status"] == "ok"
    near = abs(pred[m_pred] - tol) < 0.01 * tol or abs(pred[m_pred - 1] - tol) < 0.01 * tol
    assert info["cycles"] == m_pred or (near and abs(info["cycles"] - m_pred) == 1)
    assert info["sweeps"] == info["cycles"] * M
    assert abs(info["relres"] - pred[info["cycles"]]) <= 2e-3 * pred[info["cycles"]]


@pytest.fixture(scope="module")
def smooth():
    return workloads.smooth_3d(512, seed=0)


def test_smooth_512cube_window_bitwise(smooth):
    """Depth-5 binary64 launches (the default) with a short launch at a cycle end and a ragged
    last one: from step M - 3, 12 sweeps run as launches of 3, 5 and 4 (the z direction
    alternating between them)."""
    wl = smooth
    w, q, seq = oracle_schedule(8, wl["n"])
    M = int(np.sum(q))
    plan = srj.srj_plan(wl["n"], wl["h"], omega=w, q=q, sequence=seq)
    assert srj.srj_plan_describe(plan)["fused_sweeps"] == 5
    c = sweeps.coefficients(np.asarray(w)[seq], 3)
    b = sweeps.rhs(wl["f"], wl["h"])
    k0, n = M - 3, 12
    u = torch.from_numpy(wl["u0"]).to(DEV)
    _, launches = srj.srj_sweeps(plan, u, torch.from_numpy(wl["f"]).to(DEV), k0, n)
    assert launches == 3
    ref = sweeps.run(wl["u0"], b, c, n, k0=k0)
    assert np.array_equal(u.cpu().numpy(), ref)


def _lowprec_window(wl, ndim, w, seq, fmt, k0, n, depth):
    plan = srj.srj_plan(wl["n"], wl["h"], omega=w, q=np.bincount(seq, minlength=len(w)), sequence=seq, dtype=fmt)
    assert srj.srj_plan_describe(plan)["fused_sweeps"] == depth
    u = torch.from_numpy(wl["u0"]).to(DEV)
    srj.srj_sweeps(plan, u, torch.from_numpy(wl["f"]).to(DEV), k0, n)
    c32 = sweeps.lo_coefficients(np.asarray(w)[seq], ndim)
    x = sweeps.lo_cast(wl["u0"], fmt)
    b = sweeps.lo_cast(sweeps.rhs(wl["f"], wl["h"]), fmt)
    M = len(seq)
    for s_ in range(n):
        x = sweeps.sweep_lo(x, b, c32[(k0 + s_) % M], fmt)
    ref = sweeps.lo_widen(x, fmt)
    inner = tuple(slice(1, -1) for _ in range(ndim))
    assert np.array_equal(u.cpu().numpy()[inner], ref[inner])


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_smooth_512cube_lowprec_window_bitwise(smooth, fmt):
    """Depth-5 binary32 / bfloat16 launches at 512^3 (the benchmark's refinement sweeps):
    from step M - 3, 10 sweeps run as launches of 3, 5 and 2."""
    w, q, seq = oracle_schedule(8, smooth["n"])
    _lowprec_window(smooth, 3, w, seq, fmt, int(np.sum(q)) - 3, 10, 5)


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_blobs_4096_lowprec_window_bitwise(blobs, fmt):
    """Depth-10 binary32 / bfloat16 launches at 4096^2: from step M - 5, 25 sweeps run as
    launches of 5, 10 and 10."""
    w, q, seq = oracle_schedule(10, blobs["n"])
    _lowprec_window(blobs, 2, w, seq, fmt, int(np.sum(q)) - 5, 25, 10)


@pytest.mark.parametrize("case", ["blobs4096_P10", "adjoint2048_P9", "smooth512_P8"])
def test_product_planned_schedule_window_bitwise(case, blobs, smooth):
    """The plans the benchmark times are built by the product planner (srj_plan with P
    only).  Their weights and step order, read back through the ABI, drive the oracle on the
    same window; the GPU iterate must match it bit for bit.  The planner's weights agree with
    the oracle's optimum to 1e-8 and its counts exactly."""
    if case == "blobs4096_P10":
        wl, P, ndim = blobs, 10, 2
    elif case == "adjoint2048_P9":
        a = workloads.adjoint_2d(2048)
        wl, P, ndim = dict(n=a["n"], h=a["h"], u0=a["g"], f=a["f"]), 9, 2
    else:
        wl, P, ndim = smooth, 8, 3
    plan = srj.srj_plan(wl["n"], wl["h"], P=P)
    d = srj.srj_plan_describe(plan)
    seq = srj.srj_plan_sequence(plan)
    w = d["omega"]
    ow, oq, oseq = oracle_schedule(P, wl["n"])
    np.testing.assert_allclose(w, ow, rtol=1e-8)
    assert np.array_equal(d["q"], oq)
    M = int(d["M"])
    k0, n = (M - 7, 20) if ndim == 2 else (M - 5, 12)
    c = sweeps.coefficients(np.asarray(w)[seq], ndim)
    b = sweeps.rhs(wl["f"], wl["h"])
    u = torch.from_numpy(wl["u0"]).to(DEV)
    srj.srj_sweeps(plan, u, torch.from_numpy(wl["f"]).to(DEV), k0, n)
    ref = sweeps.run(wl["u0"], b, c, n, k0=k0)
    assert np.array_equal(u.cpu().numpy(), ref), case


def test_smooth_512cube_solves_stop_where_predicted(smooth):
    """Binary64 SRJ at 512^3 stops at the cycle the DST-mode trajectory predicts; the
    binary64 result and the binary32 / bfloat16-storage refinements (all to relres 1e-10) lie
    within cond(A) * tol of the exact discrete solution."""
    wl = smooth
    w, q, seq = oracle_schedule(8, wl["n"])
    M = int(np.sum(q))
    tol = 1e-10
    b = sweeps.rhs(wl["f"], wl["h"])
    pred = spectral.predicted_relres(wl["u0"], b, w, q, 15)
    m_pred = int(np.argmax(pred <= tol))
    assert pred[m_pred] <= tol
    ustar = spectral.exact_solve(wl["u0"], b)
    scale = float(np.max(np.abs(ustar)))
    # condition number of A: largest over smallest eigenvalue, cot^2(pi / (2 (n + 1)))
    n = wl["n"][0]
    cond = (np.cos(np.pi / (2 * (n + 1))) / np.sin(np.pi / (2 * (n + 1)))) ** 2
    f = torch.from_numpy(wl["f"]).to(DEV)
    for fmt in ("f64", "f32", "bf16"):
        plan = srj.srj_plan(wl["n"], wl["h"], omega=w, q=q, sequence=seq, dtype=fmt)
        u = torch.from_numpy(wl["u0"]).to(DEV)
        if fmt == "f64":
            info = srj.srj_solve(plan, u, f, tol, 30 * M)
            near = abs(pred[m_pred] - tol) < 0.01 * tol or abs(pred[m_pred - 1] - tol) < 0.01 * tol
            assert info["cycles"] == m_pred or (near and abs(info["cycles"] - m_pred) == 1), (info, m_pred)
            assert abs(info["relres"] - pred[info["cycles"]]) <= 2e-3 * pred[info["cycles"]]
        else:
            info = srj.srj_solve_ir(plan, u, f, tol, 1, 100)
        assert info["status"] == "ok" and info["relres"] <= tol, (fmt, info)
        err = float(np.max(np.abs(u.cpu().numpy() - ustar))) / scale
        print(f"512^3 {fmt}: sweeps {info['sweeps']}, relres {info['relres']:.3e}, "
              f"max|u - u*| / max|u*| = {err:.3e}", flush=True)
        assert err <= cond * tol, (fmt, err)
        del plan, u


def test_adjoint_2048_central_differences():
    from paper_1511_04292_amd.autograd import srj_solve_diff

    wl = workloads.adjoint_2d(2048)
    plan = srj.srj_plan((2048, 2048), wl["h"], P=9)
    f = torch.from_numpy(wl["f"]).to(DEV).requires_grad_(True)
    g = torch.from_numpy(wl["g"]).to(DEV).requires_grad_(True)
    ut = torch.from_numpy(wl["u_target"]).to(DEV)

    M = int(srj.srj_plan_describe(plan)["M"])

    def loss(ff, gg):
        u = srj_solve_diff(ff, gg, plan, tol=1e-11, max_sweeps=30 * M)
        return 0.5 * ((u - ut)[1:-1, 1:-1] ** 2).sum()

    L = loss(f, g)
    L.backward()
    rng = np.random.default_rng(2)
    for _ in range(16):
        vf = np.zeros_like(wl["f"])
        vf[1:-1, 1:-1] = rng.standard_normal((2048, 2048))
        vg = workloads.random_ring(wl["f"].shape, rng)
        eps = 1e-2
        vft, vgt = torch.from_numpy(vf).to(DEV), torch.from_numpy(vg).to(DEV)
        with torch.no_grad():
            fd = (float(loss(f + eps * vft, g + eps * vgt)) - float(loss(f - eps * vft, g - eps * vgt))) / (2 * eps)
        an = float((f.grad * vft).sum() + (g.grad * vgt).sum())
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_32768_window_sampled_bitwise():
    """32768^2 binary64, the product-planned P = 10 schedule and the default launch shape that
    bench.py times (10 sweeps per launch, automatic segment height): 14 sweeps from 4 before a
    cycle end.  After s sweeps a point depends only on points within s of it, so the oracle run
    on a crop with an s-point border (held fixed) gives the crop's inner points exactly; regions
    at the corners, on strip and segment boundaries of the fused kernel and in the middle are
    compared bit for bit."""
    n = 32768
    wl = workloads.blobs_2d_device(n, seed=0, device=DEV)
    u0, f = wl["u0"], wl["f"]
    plan = srj.srj_plan(wl["n"], wl["h"], P=10)
    d = srj.srj_plan_describe(plan)
    assert d["fused_sweeps"] == 10
    seq = srj.srj_plan_sequence(plan)
    M = int(d["M"])
    k0, nsw = M - 4, 14
    u = u0.clone()
    srj.srj_sweeps(plan, u, f, k0, nsw)
    torch.cuda.synchronize()
    c = sweeps.coefficients(np.asarray(d["omega"])[seq], 2)
    R, B = nsw, 48
    # region origins (row, column) of the interior; strips are 108 columns wide at 10 levels
    origins = [(1, 1), (n - B + 1, n - B + 1), (1, n - B + 1), (n // 2, 108 * 151 - 20),
               (4096 - 20, 108 * 7 - 30), (12345, 23456)]
    for (y, x) in origins:
        ya, yb = max(y - R, 0), min(y + B + R, n + 2)
        xa, xb = max(x - R, 0), min(x + B + R, n + 2)
        cu = u0[ya:yb, xa:xb].cpu().numpy()
        cf = f[ya:yb, xa:xb].cpu().numpy()
        ref = sweeps.run(cu, sweeps.rhs(cf, wl["h"]), c, nsw, k0=k0)
        got = u[y:y + B, x:x + B].cpu().numpy()
        assert np.array_equal(got, ref[y - ya:y - ya + B, x - xa:x - xa + B]), (y, x)
