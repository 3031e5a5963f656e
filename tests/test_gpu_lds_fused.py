"""The LDS-tiled fused sweeps (2D binary64 with unequal spacings, Neumann boundaries or a
point-wise operator with a mask), through the C ABI, against the oracle: every depth 1..8,
ragged and degenerate shapes, windows that cross a cycle end, bit for bit; and whole solves
at the default depth stop at the oracle's sweep with its iterate."""
import numpy as np
import pytest
import torch

from oracle import neumann as NE
from oracle import operator as OP
from oracle import schedule as S
from oracle import sweeps
from paper_1511_04292_amd import srj

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sched(P, km):
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    return np.asarray(o["w"]), q, S.order_balanced(o["w"], q, km)


SHAPES = [(130, 70), (64, 64), (65, 63), (1, 1), (2, 300), (300, 2), (97, 129)]


def case(kind, n, seed, km_n=None):
    """Plan, state, source, step order, oracle window and the points compared.  km_n: plan
    the schedule for the interval of that grid instead (any convergent schedule serves a
    sweep-window comparison)."""
    rng = np.random.default_rng(seed)
    full = (n[1] + 2, n[0] + 2)
    u = rng.uniform(-1, 1, full)
    f = rng.standard_normal(full)
    if kind == "spacing":
        h = (1.0 / (n[0] + 1), 0.37 / (n[1] + 1))
        w, q, seq = sched(3, S.kappa_min_dirichlet(n, h))
        p = srj.srj_plan(n, h, omega=w, q=q, sequence=seq)
        wt = sweeps.axis_weights(h, 2)
        ref = lambda nsw, k0: sweeps.run(u, sweeps.rhs(f, h), sweeps.coefficients(w[seq], 2, wt), nsw, k0=k0, wt=wt)
        return p, u, f, seq, ref, (slice(None), slice(None))
    if kind == "neumann":
        h = 1.0 / max(n)
        w, q, seq = sched(3, NE.kappa_min(km_n or n, None))
        p = srj.srj_plan(n, h, omega=w, q=q, sequence=seq, bc="neumann")
        wt = sweeps.axis_weights(h, 2)
        ref = lambda nsw, k0: NE.run(u, sweeps.rhs(f, h), sweeps.coefficients(w[seq], 2, wt), nsw, k0=k0, wt=wt)
        return p, u, f, seq, ref, (slice(1, -1), slice(1, -1))
    coef = np.zeros((5,) + full)
    coef[1:] = rng.uniform(0.2, 1.0, (4,) + full)
    coef[0] = 1.1 * coef[1:].sum(axis=0)
    mask = (rng.uniform(size=full) < 0.15).astype(np.uint8)
    w, q, seq = sched(3, 0.02)
    p = srj.srj_plan_operator(n, dev(coef), dev(mask, torch.uint8), omega=w, q=q, sequence=seq, kappa_min=0.02)
    wts, bs = OP.scale(coef, f)
    ref = lambda nsw, k0: OP.run(u, wts, bs, w[seq], nsw, k0=k0, mask=mask)
    return p, u, f, seq, ref, (slice(None), slice(None))


@pytest.mark.parametrize("kind", ["spacing", "neumann", "operator"])
@pytest.mark.parametrize("n", SHAPES)
def test_lds_fused_sweeps_bitwise(kind, n):
    if kind == "neumann" and n == (1, 1):
        pytest.skip("one Neumann cell has no nonzero symbol to plan for")
    p, u, f, seq, ref, keep = case(kind, n, 11)
    M = len(seq)
    nsw = 19
    k0 = (M - 7) % M  # the window crosses a cycle end: launches stop there and restart
    r = ref(nsw, k0)
    for T in range(1, 9):
        srj.srj_plan_set_fusion(p, T)
        ug = dev(u)
        srj.srj_sweeps(p, ug, dev(f), k0, nsw)
        got = host(ug)
        assert np.array_equal(got[keep], r[keep]), (kind, n, T)


@pytest.mark.parametrize("kind", ["spacing", "neumann", "operator"])
def test_lds_fused_solve_matches_oracle(kind):
    n = (150, 113)
    p, u, f, seq, _, keep = case(kind, n, 13)
    assert srj.srj_plan_describe(p)["fused_sweeps"] == 8
    tol = 1e-9
    if kind == "spacing":
        h = (1.0 / 151, 0.37 / 114)
        w = np.asarray(srj.srj_plan_describe(p)["omega"])
        ref = sweeps.solve(u, f, h, w[seq], tol, 10 ** 6)
    elif kind == "neumann":
        f = np.zeros_like(f)  # Eq. Laplace: a source with a nonzero mean has no solution
        w = np.asarray(srj.srj_plan_describe(p)["omega"])
        ref = NE.solve(u, f, 1.0 / 150, w[seq], tol, 10 ** 6)
    else:
        pytest.skip("operator solves at the default depth are covered by the Grad-Shafranov tests")
    ug = dev(u)
    info = srj.srj_solve(p, ug, dev(f), tol, 10 ** 6)
    assert info["status"] == ref["status"] == "ok"
    assert info["sweeps"] == ref["sweeps"]
    assert abs(info["relres"] - ref["relres"]) <= 1e-12 * ref["relres"]
    assert np.array_equal(host(ug)[keep], ref["u"][keep])


@pytest.mark.parametrize("kind", ["spacing", "neumann"])
def test_lds_fused_large_tiles_bitwise(kind):
    # grids with at least 512 tiles of 64 x 64 run the large-tile variant of the kernel
    n = (1500, 1400)
    p, u, f, seq, ref, keep = case(kind, n, 17, km_n=(400, 400))
    M = len(seq)
    k0, nsw = M - 3, 13
    r = ref(nsw, k0)
    for T in (8, 5):
        srj.srj_plan_set_fusion(p, T)
        ug = dev(u)
        srj.srj_sweeps(p, ug, dev(f), k0, nsw)
        assert np.array_equal(host(ug)[keep], r[keep]), (kind, T)
