"""Poisoned padding and run-to-run determinism (through the C ABI).

srj_plan_poison fills every plan-owned iterate, source and reduction buffer, padding and
alignment slack included, with NaN bytes.  A kernel that read any element outside the points
its stencil uses would then carry a NaN into its results; every kernel family must instead
give the same bits as on a fresh plan and as the oracle.  Repeating a run must reproduce its
bits (the 3D blocked kernel and the residual reductions synchronise through LDS barriers).
"""
import numpy as np
import pytest
import torch

from oracle import operator as OP
from oracle import schedule as S
from oracle import sweeps
from paper_1511_04292_amd import srj, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def schedule(n, P):
    km = S.kappa_min_dirichlet(n)
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    return o["w"], q, S.order_balanced(o["w"], q, km)


CASES = [
    # (name, n, dtype, fused sweeps, segment rows)
    ("tb2d_f64_T10", (301, 203), "f64", 10, 0),
    ("tb2d_f64_T7_H13", (130, 97), "f64", 7, 13),
    ("tb2d_f32_T10", (257, 120), "f32", 10, 0),
    ("tb2d_bf16_T8", (200, 99), "bf16", 8, 0),
    ("unfused2d_f64", (65, 40), "f64", 0, 0),
    ("tb3d_f64_T4", (70, 45, 33), "f64", 4, 0),
    ("tb3d_f32_T5", (57, 37, 30), "f32", 5, 0),
    ("tb3d_bf16_T3", (40, 31, 20), "bf16", 3, 0),
    ("unfused3d_f64", (33, 17, 12), "f64", 0, 0),
]


@pytest.mark.parametrize("name,n,dtype,fuse,seg", CASES, ids=[c[0] for c in CASES])
def test_poisoned_plan_sweeps_bitwise(name, n, dtype, fuse, seg):
    rng = np.random.default_rng(31)
    h = 1.0 / (max(n) + 1)
    full = tuple(x + 2 for x in reversed(n))
    u0 = workloads.random_ring(full, rng)
    u0[tuple(slice(1, -1) for _ in n)] = rng.uniform(-1, 1, tuple(x for x in reversed(n)))
    f = rng.standard_normal(full)
    w, q, seq = schedule(n, 3)
    M = len(seq)
    nsw = 2 * max(fuse, 1) + 3
    outs = []
    for poison in (False, True):
        p = srj.srj_plan(n, h, omega=w, q=q, sequence=seq, dtype=dtype)
        srj.srj_plan_set_fusion(p, fuse, seg)
        if poison:
            srj.srj_plan_poison(p)
        ug = dev(u0)
        srj.srj_sweeps(p, ug, dev(f), M - 2, nsw)
        outs.append(host(ug))
    assert np.all(np.isfinite(outs[1]))
    assert np.array_equal(outs[0], outs[1])
    if dtype == "f64":
        c = sweeps.coefficients(np.asarray(w)[seq], len(n))
        assert np.array_equal(outs[1], sweeps.run(u0, sweeps.rhs(f, h), c, nsw, k0=M - 2))


@pytest.mark.parametrize("kind", ["resident", "tb2d", "unfused2d", "ir_f32", "residual"])
def test_poisoned_plan_solves_bitwise(kind):
    rng = np.random.default_rng(8)
    n = (50, 41) if kind == "resident" else (120, 97)
    h = 1.0 / (max(n) + 1)
    full = (n[1] + 2, n[0] + 2)
    u0 = workloads.random_ring(full, rng)
    f = rng.standard_normal(full)
    w, q, seq = schedule(n, 4)
    wseq = np.asarray(w)[seq]
    p = srj.srj_plan(n, h, omega=w, q=q, sequence=seq, dtype="f32" if kind == "ir_f32" else "f64")
    if kind == "unfused2d":
        srj.srj_plan_set_fusion(p, 0)
    assert srj.srj_plan_describe(p)["resident"] == (1 if kind == "resident" else 0)
    srj.srj_plan_poison(p)
    ug = dev(u0)
    if kind == "residual":
        r = torch.zeros_like(ug)
        got = srj.srj_residual(p, ug, dev(f), r)
        b = sweeps.rhs(f, h)
        r2, rmax = sweeps.residual_norms(u0, b)
        assert got["linf"] == rmax and np.array_equal(host(r), sweeps.residual_field(u0, b))
        return
    if kind == "ir_f32":
        info = srj.srj_solve_ir(p, ug, dev(f), 1e-10, 1, 100)
        ref = sweeps.solve_ir(u0, f, h, wseq, 1e-10, 1, 100, "f32")
    else:
        info = srj.srj_solve(p, ug, dev(f), 1e-10, 10 ** 6)
        ref = sweeps.solve(u0, f, h, wseq, 1e-10, 10 ** 6)
    assert info["status"] == "ok" and info["sweeps"] == ref["sweeps"]
    assert np.array_equal(host(ug), ref["u"])


@pytest.mark.parametrize("nd", [2, 3])
def test_poisoned_operator_plan_bitwise(nd):
    n = (45, 38) if nd == 2 else (17, 13, 11)
    shape = tuple(x + 2 for x in reversed(n))
    rng = np.random.default_rng(6)
    coef = np.zeros((2 * nd + 1,) + shape)
    coef[1:] = rng.uniform(0.2, 1.0, (2 * nd,) + shape)
    coef[0] = 1.1 * coef[1:].sum(axis=0)
    u = rng.uniform(-1, 1, shape)
    f = rng.standard_normal(shape)
    mask = (rng.uniform(size=shape) < 0.2).astype(np.uint8)
    km = 0.05
    o = S.optimal(3, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    nsw = len(seq) + 4
    outs = []
    for poison in (False, True):
        p = srj.srj_plan_operator(n, dev(coef), torch.from_numpy(mask).to(DEV), omega=o["w"], q=q, sequence=seq,
                                  kappa_min=km)
        if poison:
            srj.srj_plan_poison(p)
        ug = dev(u)
        srj.srj_sweeps(p, ug, dev(f), 2, nsw)
        outs.append(host(ug))
    wts, bs = OP.scale(coef, f)
    ref = OP.run(u, wts, bs, np.asarray(o["w"])[seq], nsw, k0=2, mask=mask)
    assert np.all(np.isfinite(outs[1])) and np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[1], ref)


def test_repeated_runs_are_bitwise_identical():
    # blocked 3D (LDS exchange and a barrier per plane) and 2D launches at sizes that fill the
    # device several times, run twice from the same state
    rng = np.random.default_rng(12)
    for n, fuse in (((160, 150, 140), 4), ((1500, 1300), 10)):
        full = tuple(x + 2 for x in reversed(n))
        u0 = rng.uniform(-1, 1, full)
        f = rng.standard_normal(full)
        p = srj.srj_plan(n, 1.0 / (max(n) + 1), P=5)
        srj.srj_plan_set_fusion(p, fuse)
        runs = []
        for _ in range(2):
            ug = dev(u0)
            srj.srj_sweeps(p, ug, dev(f), 0, 6 * fuse + 1)
            runs.append(host(ug))
        assert np.array_equal(runs[0], runs[1]), n
        nr = [srj.srj_residual(p, dev(runs[0]), dev(f)) for _ in range(2)]
        assert nr[0] == nr[1]
