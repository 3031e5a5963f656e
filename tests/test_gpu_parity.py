"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

FP64 sweeps use the same association as the oracle and no fused multiply-add, so the
iterates must be bit-identical; residual norms are sums in a different order and are
compared to 1e-12 relative.
"""
import math

import numpy as np
import pytest
import torch

from oracle import schedule as S
from oracle import spectral, sweeps
from paper_1511_04292_amd import srj, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_case(shape_interior, seed):
    full = tuple(n + 2 for n in reversed(shape_interior))
    u = workloads.random_state(full, seed)
    f = workloads.random_state(full, seed + 1000)
    return u, f


def oracle_schedule(P, n_interior, ordering=0):
    km = S.kappa_min_dirichlet(n_interior)
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km) if ordering == 0 else S.order_even(q)
    return o["w"], q, seq


_SCHED = {}


def shared_schedule(P=3, n_ref=(300, 300)):
    """Oracle schedule optimised for a 300 x 300 grid; convergent on every smaller grid
    because their spectra lie inside its interval."""
    key = (P, n_ref)
    if key not in _SCHED:
        _SCHED[key] = oracle_schedule(P, n_ref)
    return _SCHED[key]


def big_first(P=3):
    """The shared schedule rotated so that its largest weight is applied first."""
    w, q, seq = shared_schedule(P)
    k = int(np.argmax(np.asarray(seq) == 0))
    return w, q, np.roll(seq, -k)


def explicit_plan(n, h, w, q, seq, dtype="f64", fuse=None, seg_rows=0):
    p = srj.srj_plan(n, h, omega=w, q=q, sequence=seq, dtype=dtype)
    if fuse is not None:
        srj.srj_plan_set_fusion(p, fuse, seg_rows)
    return p


# ------------------------------------------------------------------ single sweeps

@pytest.mark.parametrize("n", [(1, 1), (2, 3), (67, 45), (130, 257), (1, 9), (300, 2)])
def test_single_sweep_2d_bitwise(n):
    h = 1.0 / (max(n) + 1)
    u, f = rand_case(n, 1)
    w, q, seq = big_first()
    p = explicit_plan(n, h, w, q, seq, fuse=0)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 0, 1)
    ref = sweeps.sweep(u, sweeps.rhs(f, h), w[0] / 4.0)
    assert np.array_equal(host(ug), ref)


@pytest.mark.parametrize("n", [(1, 1, 1), (5, 7, 3), (33, 17, 40), (64, 1, 9)])
def test_single_sweep_3d_bitwise(n):
    h = 1.0 / (max(n) + 1)
    u, f = rand_case(n, 2)
    w, q, seq = big_first()
    p = explicit_plan(n, h, w, q, seq)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 0, 1)
    ref = sweeps.sweep(u, sweeps.rhs(f, h), w[0] / 6.0)
    assert np.array_equal(host(ug), ref)


# ------------------------------------------------------- temporally blocked sweeps

@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
@pytest.mark.parametrize("n", [(300, 200), (129, 150), (2, 2), (1, 70), (250, 1)])
def test_fused_sweeps_bitwise(T, n):
    h = 1.0 / (max(n) + 1)
    u, f = rand_case(n, 3)
    w, q, seq = shared_schedule()
    nsweeps = 2 * len(seq) + 5  # crosses cycle ends and leaves a ragged last launch
    p = explicit_plan(n, h, w, q, seq, fuse=T)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 3, nsweeps)
    c = sweeps.coefficients(np.array(w)[seq], 2)
    ref = sweeps.run(u, sweeps.rhs(f, h), c, nsweeps, k0=3)
    assert np.array_equal(host(ug), ref)


@pytest.mark.parametrize("T,H", [(8, 8), (8, 13), (3, 100), (5, 1), (8, 512), (10, 10), (10, 77), (9, 5), (10, 203)])
def test_fused_segment_heights_bitwise(T, H):
    n = (300, 203)
    h = 1.0 / 301
    u, f = rand_case(n, 9)
    w, q, seq = shared_schedule()
    nsweeps = 3 * T + 1
    p = explicit_plan(n, h, w, q, seq, fuse=T, seg_rows=H)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 0, nsweeps)
    c = sweeps.coefficients(np.array(w)[seq], 2)
    ref = sweeps.run(u, sweeps.rhs(f, h), c, nsweeps)
    assert np.array_equal(host(ug), ref)


def test_fused_stream_direction_alternates_without_changing_results():
    """The plan alternates the stream direction of its segments from launch to launch; calls
    that start on either parity give the oracle's iterate bit for bit."""
    n = (257, 190)
    h = 1.0 / 258
    u, f = rand_case(n, 12)
    w, q, seq = shared_schedule()
    c = sweeps.coefficients(np.array(w)[seq], 2)
    b = sweeps.rhs(f, h)
    for first in (10, 20, 7):  # one, two or one partial launch before the second call
        p = explicit_plan(n, h, w, q, seq, fuse=10, seg_rows=40)
        ug = dev(u)
        fg = dev(f)
        srj.srj_sweeps(p, ug, fg, 0, first)
        srj.srj_sweeps(p, ug, fg, first, 33)
        ref = sweeps.run(u, b, c, first + 33)
        assert np.array_equal(host(ug), ref), first


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("n", [(70, 45, 33), (5, 7, 3), (130, 40, 9), (1, 1, 1), (64, 1, 20), (57, 37, 70)])
def test_fused3d_sweeps_bitwise(T, n):
    """3D x-y tiles streamed in z, T sweeps per launch: bit-identical to the oracle's sweeps
    (tiles and z runs ragged, cycle ends crossed, last launch shorter)."""
    h = 1.0 / (max(n) + 1)
    u, f = rand_case(n, 5)
    w, q, seq = shared_schedule()
    nsweeps = 2 * len(seq) + 3
    p = explicit_plan(n, h, w, q, seq, fuse=T)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 1, nsweeps)
    c = sweeps.coefficients(np.array(w)[seq], 3)
    ref = sweeps.run(u, sweeps.rhs(f, h), c, nsweeps, k0=1)
    assert np.array_equal(host(ug), ref)


def test_fused_equals_unfused_on_gpu():
    n = (517, 389)
    h = 1.0 / 518
    u, f = rand_case(n, 4)
    w, q, seq = oracle_schedule(5, n)
    outs = []
    for T in (0, 8, 10):
        p = explicit_plan(n, h, w, q, seq, fuse=T)
        ug = dev(u)
        srj.srj_sweeps(p, ug, dev(f), 0, 2 * int(np.sum(q)) + 3)
        outs.append(host(ug))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


# ------------------------------------------------------------------ residuals

@pytest.mark.parametrize("n", [(64, 64), (123, 77), (9, 10, 11)])
def test_residual_norms(n):
    h = 1.0 / (max(n) + 1)
    u, f = rand_case(n, 5)
    p = srj.srj_plan(n, h, omega=[1.0], q=[1])
    r = torch.zeros_like(dev(u))
    got = srj.srj_residual(p, dev(u), dev(f), r)
    b = sweeps.rhs(f, h)
    r2, rmax = sweeps.residual_norms(u, b)
    bt2 = sweeps.source_norm2(u, b)
    assert math.isclose(got["l2"], math.sqrt(r2), rel_tol=1e-12)
    assert got["linf"] == rmax
    assert math.isclose(got["source_l2"], math.sqrt(bt2), rel_tol=1e-12)
    assert np.array_equal(host(r), sweeps.residual_field(u, b))


# ------------------------------------------------------------------ solves

def test_solve_small_2d_srj_matches_oracle():
    wl = workloads.small_2d(64, seed=0)
    w, q, seq = oracle_schedule(2, wl["n"])
    wseq = np.array(w)[seq]
    ref = sweeps.solve(wl["u0"], wl["f"], wl["h"], wseq, 1e-10, 10 ** 5)
    for fuse in (None, 0, 8):  # None: the default, one workgroup with the grid in LDS
        p = explicit_plan(wl["n"], wl["h"], w, q, seq, fuse=fuse)
        assert srj.srj_plan_describe(p)["resident"] == (1 if fuse is None else 0)
        ug = dev(wl["u0"])
        info = srj.srj_solve(p, ug, dev(wl["f"]), 1e-10, 10 ** 5)
        assert info["status"] == "ok" and ref["status"] == "ok"
        assert info["sweeps"] == ref["sweeps"]
        assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
        assert np.array_equal(host(ug), ref["u"])
    # the converged iterate is within the conditioning bound of the exact discrete solution
    us = spectral.exact_solve(wl["u0"], sweeps.rhs(wl["f"], wl["h"]))
    cond = math.cos(math.pi / 130) ** 2 / math.sin(math.pi / 130) ** 2
    assert np.max(np.abs(ref["u"] - us)) <= cond * 1e-10 * np.max(np.abs(us))


def test_solve_jacobi_matches_oracle():
    wl = workloads.small_2d(20, seed=1)
    ref = sweeps.solve(wl["u0"], wl["f"], wl["h"], [1.0], 1e-6, 10 ** 5)
    for resident in (True, False):
        p = srj.srj_plan(wl["n"], wl["h"], omega=[1.0], q=[1])
        if not resident:
            srj.srj_plan_set_fusion(p, 10)
        ug = dev(wl["u0"])
        info = srj.srj_solve(p, ug, dev(wl["f"]), 1e-6, 10 ** 5)
        assert info["sweeps"] == ref["sweeps"]
        assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
        assert np.array_equal(host(ug), ref["u"])


@pytest.mark.parametrize("case", ["srj2d_unfused", "jacobi2d_blocked", "jacobi3d_blocked", "srj3d_unfused"])
def test_fused_cycle_check_matches_oracle(case):
    """Binary64 plans that sweep one step per launch, and single-sweep cycles, take each
    cycle's check from the cycle's first sweep: the stopping sweep, the relres and the
    returned (checked, not advanced) state are the oracle's."""
    rng = np.random.default_rng(23)
    n = {"srj2d_unfused": (101, 70), "jacobi2d_blocked": (100, 70),
         "jacobi3d_blocked": (12, 11, 10), "srj3d_unfused": (19, 13, 11)}[case]
    h = 1.0 / (max(n) + 1)
    full = tuple(x + 2 for x in reversed(n))
    u0 = workloads.random_ring(full, rng)
    f = rng.standard_normal(full)
    if case.startswith("jacobi"):
        w, q, seq, tol, fuse = [1.0], [1], [0], 1e-2, (10 if len(n) == 2 else 4)
    else:
        w, q, seq = oracle_schedule(3, n)
        tol, fuse = 1e-10, 0
    ref = sweeps.solve(u0, f, h, np.asarray(w)[seq], tol, 10 ** 6)
    p = explicit_plan(n, h, w, q, seq, fuse=fuse)
    assert srj.srj_plan_describe(p)["resident"] == 0
    ug = dev(u0)
    info = srj.srj_solve(p, ug, dev(f), tol, 10 ** 6)
    assert info["status"] == ref["status"] == "ok"
    assert info["sweeps"] == ref["sweeps"] > 0
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
    assert np.array_equal(host(ug), ref["u"])
    # a sweep budget that ends inside the next cycle: the last checked state comes back
    M = len(seq)
    cap = max(ref["sweeps"] - M, 0) + (M - 1 if M > 1 else 0)
    ref2 = sweeps.solve(u0, f, h, np.asarray(w)[seq], tol, cap)
    ug2 = dev(u0)
    info2 = srj.srj_solve(p, ug2, dev(f), tol, cap)
    assert ref2["status"] == "noconv" and info2["status"] == "enoconv"
    assert info2["sweeps"] == ref2["sweeps"]
    assert np.array_equal(host(ug2), ref2["u"])


@pytest.mark.parametrize("n,h", [((79, 79), None), ((1, 1), None), ((3, 200), None), ((61, 47), (1.0 / 62, 1.0 / 20))])
def test_resident_small_solve_matches_oracle(n, h):
    """Grids up to 6656 points with the ring are solved in one workgroup with the grid in LDS:
    the same stopping sweep and iterate as the oracle (equal and unequal spacings, the largest
    such square, degenerate shapes)."""
    hh = h if h is not None else 1.0 / (max(n) + 1)
    rng = np.random.default_rng(17)
    full = (n[1] + 2, n[0] + 2)
    u0 = workloads.random_ring(full, rng)
    f = rng.standard_normal(full)
    km = S.kappa_min_dirichlet(n, h)
    o = S.optimal(3, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    ref = sweeps.solve(u0, f, hh, np.asarray(o["w"])[seq], 1e-11, 10 ** 6)
    p = srj.srj_plan(n, hh, omega=o["w"], q=q, sequence=seq)
    assert srj.srj_plan_describe(p)["resident"] == 1
    ug = dev(u0)
    info = srj.srj_solve(p, ug, dev(f), 1e-11, 10 ** 6)
    assert info["status"] == ref["status"] == "ok" and info["sweeps"] == ref["sweeps"]
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * max(ref["relres"], 1e-300)
    assert np.array_equal(host(ug), ref["u"])
    big = srj.srj_plan((80, 80), 1.0 / 81, omega=[1.0], q=[1])
    assert srj.srj_plan_describe(big)["resident"] == 0


def test_solve_3d_matches_oracle():
    n = (20, 17, 23)
    h = 1.0 / 24
    rng = np.random.default_rng(7)
    full = tuple(x + 2 for x in reversed(n))
    u0 = workloads.random_ring(full, rng)
    f = rng.standard_normal(full)
    w, q, seq = oracle_schedule(4, n)
    wseq = np.array(w)[seq]
    ref = sweeps.solve(u0, f, h, wseq, 1e-10, 10 ** 5)
    p = explicit_plan(n, h, w, q, seq)
    ug = dev(u0)
    info = srj.srj_solve(p, ug, dev(f), 1e-10, 10 ** 5)
    assert info["sweeps"] == ref["sweeps"]
    assert np.array_equal(host(ug), ref["u"])


def test_product_planner_plan_solves_cfg_small():
    # a plan that runs its own optimiser and ordering converges and reports its schedule
    wl = workloads.small_2d(64, seed=0)
    p = srj.srj_plan(wl["n"], wl["h"], P=2)
    d = srj.srj_plan_describe(p)
    assert d["M"] == int(np.sum(d["q"])) and d["gamma_q_max"] < 1
    ug = dev(wl["u0"])
    info = srj.srj_solve(p, ug, dev(wl["f"]), 1e-10, 10 ** 5)
    assert info["status"] == "ok" and info["relres"] <= 1e-10


# ----------------------------------------------------------- reduced precision

@pytest.mark.parametrize("fmt", ["f32", "bf16"])
@pytest.mark.parametrize("fuse", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_lowprec_sweeps_bitwise(fmt, fuse):
    n = (200, 131)
    h = 1.0 / 201
    u, f = rand_case(n, 8)
    w, q, seq = big_first()
    nsw = 17
    p = explicit_plan(n, h, w, q, seq, dtype=fmt, fuse=fuse)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 0, nsw)
    c32 = sweeps.lo_coefficients(np.array(w)[seq], 2)
    x = sweeps.lo_cast(u, fmt)
    b = sweeps.lo_cast(sweeps.rhs(f, h), fmt)
    for s in range(nsw):
        x = sweeps.sweep_lo(x, b, c32[s % len(seq)], fmt)
    ref = sweeps.lo_widen(x, fmt)
    got = host(ug)
    inner = (slice(1, -1), slice(1, -1))
    assert np.array_equal(got[inner], ref[inner])


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_ir_matches_oracle(fmt):
    wl = workloads.small_2d(63, seed=4)
    w, q, seq = oracle_schedule(4, wl["n"])
    wseq = np.array(w)[seq]
    ref = sweeps.solve_ir(wl["u0"], wl["f"], wl["h"], wseq, 1e-10, 1, 60, fmt)
    p = explicit_plan(wl["n"], wl["h"], w, q, seq, dtype=fmt)
    ug = dev(wl["u0"])
    info = srj.srj_solve_ir(p, ug, dev(wl["f"]), 1e-10, 1, 60)
    assert ref["status"] == "ok" and info["status"] == "ok"
    assert info["cycles"] == ref["outer"]
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
    assert np.array_equal(host(ug), ref["u"])


@pytest.mark.parametrize("ndim", [2, 3])
def test_ir_f64_matches_oracle(ndim):
    """Refinement on a binary64 plan: its inner right-hand side must not overwrite b (one
    inner cycle per outer step, so several outer steps are needed)."""
    if ndim == 2:
        wl = workloads.small_2d(47, seed=5)
        n, h, u0, f = wl["n"], wl["h"], wl["u0"], wl["f"]
    else:
        n, h = (13, 16, 11), 1.0 / 17
        rng = np.random.default_rng(33)
        full = tuple(x + 2 for x in reversed(n))
        u0 = workloads.random_ring(full, rng)
        f = rng.standard_normal(full)
    w, q, seq = oracle_schedule(3, n)
    wseq = np.array(w)[seq]
    ref = sweeps.solve_ir(u0, f, h, wseq, 1e-10, 1, 200, "f64")
    assert ref["status"] == "ok" and ref["outer"] >= 2
    p = explicit_plan(n, h, w, q, seq, dtype="f64")
    ug = dev(u0)
    info = srj.srj_solve_ir(p, ug, dev(f), 1e-10, 1, 200)
    assert info["status"] == "ok" and info["relres"] <= 1e-10
    assert info["cycles"] == ref["outer"]
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
    assert np.array_equal(host(ug), ref["u"])
    # and the same state as the plain solve reaches, to the solve's tolerance
    plain = sweeps.solve(u0, f, h, wseq, 1e-10, 10 ** 6)
    assert np.max(np.abs(ref["u"] - plain["u"])) <= 1e-6 * np.max(np.abs(plain["u"]))


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
@pytest.mark.parametrize("fuse", [0, 1, 2, 3, 4, 5])
def test_lowprec_sweeps_3d_bitwise(fmt, fuse):
    n = (70, 37, 29)
    h = 1.0 / 71
    u, f = rand_case(n, 18)
    w, q, seq = big_first()
    nsw = 9
    p = explicit_plan(n, h, w, q, seq, dtype=fmt, fuse=fuse)
    ug = dev(u)
    srj.srj_sweeps(p, ug, dev(f), 0, nsw)
    c32 = sweeps.lo_coefficients(np.array(w)[seq], 3)
    x = sweeps.lo_cast(u, fmt)
    b = sweeps.lo_cast(sweeps.rhs(f, h), fmt)
    for s in range(nsw):
        x = sweeps.sweep_lo(x, b, c32[s % len(seq)], fmt)
    ref = sweeps.lo_widen(x, fmt)
    got = host(ug)
    inner = (slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.array_equal(got[inner], ref[inner])


@pytest.mark.parametrize("fmt", ["f32", "bf16"])
def test_ir_3d_matches_oracle(fmt):
    n = (21, 18, 15)
    h = 1.0 / 22
    rng = np.random.default_rng(31)
    full = tuple(x + 2 for x in reversed(n))
    u0 = workloads.random_ring(full, rng)
    f = rng.standard_normal(full)
    w, q, seq = oracle_schedule(4, n)
    wseq = np.array(w)[seq]
    ref = sweeps.solve_ir(u0, f, h, wseq, 1e-10, 1, 60, fmt)
    p = explicit_plan(n, h, w, q, seq, dtype=fmt)
    ug = dev(u0)
    info = srj.srj_solve_ir(p, ug, dev(f), 1e-10, 1, 60)
    assert ref["status"] == "ok" and info["status"] == "ok"
    assert info["cycles"] == ref["outer"]
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
    assert np.array_equal(host(ug), ref["u"])


# ------------------------------------------------------------------ error paths

def test_errors():
    with pytest.raises(srj.SrjError) as e:
        srj.srj_plan((0, 5), 0.1, omega=[1.0], q=[1])
    assert e.value.status == 1
    with pytest.raises(srj.SrjError) as e:
        srj.srj_plan((5, 5), 0.1, omega=[3.0], q=[1])  # |1 - 3 kappa| > 1 near kappa = 2
    assert e.value.status == 4
    with pytest.raises(srj.SrjError) as e:
        srj.srj_plan((5, 5), 0.1, omega=[1.0, 2.0], q=[1, 1])  # not descending
    assert e.value.status == 1
    wl = workloads.small_2d(16, seed=2)
    p = srj.srj_plan(wl["n"], wl["h"], omega=[1.0], q=[1])
    info = srj.srj_solve(p, dev(wl["u0"]), dev(wl["f"]), 1e-10, 10)
    assert info["status"] == "enoconv" and info["sweeps"] == 10
    f = wl["f"].copy()
    f[4, 4] = np.nan
    info = srj.srj_solve(p, dev(wl["u0"]), dev(f), 1e-10, 10)
    assert info["status"] == "ediverged"
    z = np.zeros_like(wl["f"])
    ug = dev(z + 0.0)
    ug[3, 3] = 7.0
    info = srj.srj_solve(p, ug, dev(z), 1e-10, 10)
    assert info["status"] == "ok" and info["sweeps"] == 0 and float(ug.abs().max()) == 0.0
    # fusion depths: at most 10 in 2D (the default), 5 in 3D (the default is 5, 4 or 3, from a
    # model of the launch shape: 4 for this small grid);
    # segment heights non-negative
    assert srj.srj_plan_describe(p)["fused_sweeps"] == 10
    with pytest.raises(srj.SrjError) as e:
        srj.srj_plan_set_fusion(p, 11)
    assert e.value.status == 1
    with pytest.raises(srj.SrjError) as e:
        srj.srj_plan_set_fusion(p, 8, -1)
    assert e.value.status == 1
    p3 = srj.srj_plan((6, 5, 4), 1.0 / 7, omega=[1.0], q=[1])
    assert srj.srj_plan_describe(p3)["fused_sweeps"] == 4
    with pytest.raises(srj.SrjError) as e:
        srj.srj_plan_set_fusion(p3, 6)
    assert e.value.status == 1
    srj.srj_plan_set_fusion(p3, 0)
    assert srj.srj_plan_describe(p3)["fused_sweeps"] == 0


def test_store_hint_follows_the_working_set():
    """Fused 2D binary64 plans store with the non-temporal hint when input, output and b exceed
    the 256 MiB memory-side cache but fit in twice it (4096^2 yes; 2048^2 and 8192^2 no); the
    flag is reported for 2D binary64 plans only (3D binary64 always takes the hint, the other
    formats never)."""
    assert srj.srj_plan_describe(srj.srj_plan((4096, 4096), 1.0 / 4097, omega=[1.0], q=[1]))["store_nt"] == 1
    assert srj.srj_plan_describe(srj.srj_plan((8192, 8192), 1.0 / 8193, omega=[1.0], q=[1]))["store_nt"] == 0
    assert srj.srj_plan_describe(srj.srj_plan((2048, 2048), 1.0 / 2049, omega=[1.0], q=[1]))["store_nt"] == 0
    assert srj.srj_plan_describe(srj.srj_plan((64, 48), 1.0 / 65, omega=[1.0], q=[1]))["store_nt"] == 0
    assert srj.srj_plan_describe(srj.srj_plan((4096, 4096), 1.0 / 4097, omega=[1.0], q=[1],
                                              dtype="f32"))["store_nt"] == 0
    assert srj.srj_plan_describe(srj.srj_plan((64, 64, 64), 1.0 / 65, omega=[1.0], q=[1]))["store_nt"] == 0
    # plans that run the LDS-tiled kernel instead report 0
    assert srj.srj_plan_describe(srj.srj_plan((64, 48), (1.0 / 65, 0.5 / 49), omega=[1.0], q=[1]))["store_nt"] == 0
    assert srj.srj_plan_describe(srj.srj_plan((64, 48), 1.0 / 64, omega=[1.0], q=[1], bc="neumann"))["store_nt"] == 0


def test_nan_source_diverges_on_every_path():
    """A NaN in the source makes every solve path report SRJ_EDIVERGED at its first check:
    the blocked 2D kernel, one sweep per launch (check fused into the cycle's first sweep),
    the LDS-tiled kernels (unequal spacings, Neumann, operator), 3D, and the batch, where only
    the problem holding the NaN fails."""
    n = (90, 80)
    rng = np.random.default_rng(5)
    full = (n[1] + 2, n[0] + 2)
    u0 = np.zeros(full)
    f = rng.standard_normal(full)
    f[40, 33] = np.nan
    plans = []
    p = srj.srj_plan(n, 1.0 / 91, P=3)
    plans.append(("blocked", p))
    p = srj.srj_plan(n, 1.0 / 91, P=3)
    srj.srj_plan_set_fusion(p, 0)
    plans.append(("one sweep per launch", p))
    plans.append(("lds spacing", srj.srj_plan(n, (1.0 / 91, 0.5 / 81), P=3)))
    plans.append(("lds neumann", srj.srj_plan(n, 1.0 / 90, P=3, bc="neumann")))
    coef = np.zeros((5,) + full)
    coef[1:] = 1.0
    coef[0] = 4.5
    plans.append(("lds operator", srj.srj_plan_operator(n, dev(coef), None, P=3, kappa_min=0.01)))
    for name, p in plans:
        info = srj.srj_solve(p, dev(u0), dev(f), 1e-10, 10 ** 5)
        assert info["status"] == "ediverged", (name, info)
    n3 = (20, 18, 16)
    f3 = rng.standard_normal((18, 20, 22))
    f3[5, 6, 7] = np.nan
    p3 = srj.srj_plan(n3, 1.0 / 21, P=3)
    info = srj.srj_solve(p3, dev(np.zeros_like(f3)), dev(f3), 1e-10, 10 ** 5)
    assert info["status"] == "ediverged"
    probs = [dict(n=(40, 40), h=1.0 / 41, P=3), dict(n=(50, 45), h=1.0 / 51, P=3)]
    fa = rng.standard_normal((42, 42))
    fb = rng.standard_normal((47, 52))
    fb[10, 10] = np.nan
    b = srj.srj_batch_plan(probs, dtype="f32")
    infos, _ = srj.srj_batch_solve(b, [dev(np.zeros((42, 42))), dev(np.zeros((47, 52)))], [dev(fa), dev(fb)],
                                   1e-10, 1, 200)
    assert infos[0]["status"] == "ok" and infos[1]["status"] == "ediverged"
