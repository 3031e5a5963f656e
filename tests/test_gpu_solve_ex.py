"""srj_solve_ex (relres history, resumed solves) and srj_plan_tune_cached, through the C ABI.

The history is the relres at every check (Sec. 4's residual curves), compared with the
oracle's to 1e-12 relative; a solve resumed from a checkpoint taken mid-cycle must stop at
the same sweep and return the same bits as the uninterrupted one.
"""
import os

import numpy as np
import pytest
import torch

from oracle import neumann as NE
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


def case(kind, seed=5):
    rng = np.random.default_rng(seed)
    n = {"tb2d": (150, 131), "unfused2d": (90, 77), "small2d": (40, 33), "tb3d": (21, 18, 16)}[kind]
    h = 1.0 / (max(n) + 1)
    full = tuple(x + 2 for x in reversed(n))
    u0 = workloads.random_ring(full, rng)
    f = rng.standard_normal(full)
    km = S.kappa_min_dirichlet(n)
    o = S.optimal(4 if len(n) == 2 else 3, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    p = srj.srj_plan(n, h, omega=o["w"], q=q, sequence=seq)
    if kind == "unfused2d":
        srj.srj_plan_set_fusion(p, 0)
    return p, u0, f, h, np.asarray(o["w"])[seq]


@pytest.mark.parametrize("kind", ["tb2d", "unfused2d", "small2d", "tb3d"])
def test_history_matches_oracle(kind):
    p, u0, f, h, wseq = case(kind)
    ref = sweeps.solve(u0, f, h, wseq, 1e-10, 10 ** 6, history=True)
    ug = dev(u0)
    info = srj.srj_solve_ex(p, ug, dev(f), 1e-10, 10 ** 6, history_cap=10 ** 4)
    assert info["status"] == ref["status"] == "ok"
    assert info["sweeps"] == ref["sweeps"]
    assert info["checks"] == len(ref["history"]) == info["cycles"] + 1
    np.testing.assert_allclose(info["history"], ref["history"], rtol=1e-12, atol=0)
    assert np.array_equal(host(ug), ref["u"])
    # a short buffer keeps the first entries and still counts every check
    ug = dev(u0)
    info3 = srj.srj_solve_ex(p, ug, dev(f), 1e-10, 10 ** 6, history_cap=3)
    assert info3["checks"] == info["checks"] and info3["history"] == info["history"][:3]


@pytest.mark.parametrize("kind", ["tb2d", "unfused2d", "tb3d"])
def test_resumed_solve_equals_uninterrupted(kind):
    p, u0, f, h, wseq = case(kind)
    M = len(wseq)
    ref = sweeps.solve(u0, f, h, wseq, 1e-10, 10 ** 6, history=True)
    assert ref["sweeps"] > 2 * M
    kc = M + M // 2 + 1  # a checkpoint in the middle of the second cycle
    uc = dev(u0)
    srj.srj_sweeps(p, uc, dev(f), 0, kc)
    c = sweeps.coefficients(wseq, u0.ndim)
    assert np.array_equal(host(uc), sweeps.run(u0, sweeps.rhs(f, h), c, kc))
    info = srj.srj_solve_ex(p, uc, dev(f), 1e-10, 10 ** 6, start_offset=kc % M, history_cap=10 ** 4)
    assert info["status"] == "ok"
    assert kc + info["sweeps"] == ref["sweeps"]
    assert np.array_equal(host(uc), ref["u"])
    # its checks are the uninterrupted solve's from the end of the checkpoint's cycle on
    np.testing.assert_allclose(info["history"], ref["history"][2:], rtol=1e-12, atol=0)
    # a budget that ends before the started cycle does: u comes back unchanged
    ub = dev(u0)
    srj.srj_sweeps(p, ub, dev(f), 0, kc)
    before = host(ub).copy()
    info2 = srj.srj_solve_ex(p, ub, dev(f), 1e-10, M - kc % M - 1, start_offset=kc % M)
    assert info2["status"] == "enoconv" and info2["sweeps"] == 0 and info2["checks"] == 0
    assert np.array_equal(host(ub), before)
    with pytest.raises(srj.SrjError):
        srj.srj_solve_ex(p, ub, dev(f), 1e-10, 10, start_offset=M)


def test_neumann_history_matches_oracle():
    # Neumann plans measure relres against the residual of the state they are given
    N = 64
    rng = np.random.default_rng(3)
    u0 = rng.uniform(-1, 1, (N + 2, N + 2))
    f = np.zeros_like(u0)
    km = S.kappa_min_neumann(N)
    o = S.optimal(3, km)
    q = S.q_floor(o["beta"])
    seq = S.order_balanced(o["w"], q, km)
    wseq = np.asarray(o["w"])[seq]
    ref = NE.solve(u0, f, 1.0 / N, wseq, 1e-8, 10 ** 6, history=True)
    p = srj.srj_plan((N, N), 1.0 / N, omega=o["w"], q=q, sequence=seq, bc="neumann")
    ug = dev(u0)
    info = srj.srj_solve_ex(p, ug, dev(f), 1e-8, 10 ** 6, history_cap=10 ** 4)
    assert info["status"] == ref["status"] == "ok" and info["sweeps"] == ref["sweeps"]
    np.testing.assert_allclose(info["history"], ref["history"], rtol=1e-12, atol=0)
    assert np.array_equal(host(ug)[1:-1, 1:-1], ref["u"][1:-1, 1:-1])


def test_tune_cache_roundtrip(tmp_path):
    path = str(tmp_path / "srj_tune.txt")
    n = (700, 650)
    a = srj.srj_plan(n, 1.0 / 701, P=6)
    t1 = srj.srj_plan_tune_cached(a, path)
    assert t1["candidates"] > 0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("srj-tune-v2 ")
    b = srj.srj_plan(n, 1.0 / 701, P=6)
    t2 = srj.srj_plan_tune_cached(b, path)
    assert t2["candidates"] == 0
    assert (t2["fused_sweeps"], t2["seg_rows"]) == (t1["fused_sweeps"], t1["seg_rows"])
    db = srj.srj_plan_describe(b)
    assert db["fused_sweeps"] == t1["fused_sweeps"]
    # another grid misses and appends; a line naming a shape the plan cannot run is skipped
    c = srj.srj_plan((300, 200), 1.0 / 301, P=5)
    with open(path, "a") as fp:
        key = lines[0].split()[1:12]
        key[3:5] = ["300", "200"]
        key[10] = str(srj.srj_plan_describe(c)["M"])
        fp.write("srj-tune-v2 " + " ".join(key) + " 7 5 1.0\n")
        fp.write("garbage line\n")
    t3 = srj.srj_plan_tune_cached(c, path)
    assert t3["candidates"] > 0 and t3["fused_sweeps"] != 7
    assert len(open(path).read().splitlines()) == 4
    # results do not depend on the launch shape the cache picks
    wl = workloads.batch_problem(300, seed=1)
    u0 = np.zeros((202, 302))
    f = np.random.default_rng(2).standard_normal((202, 302))
    ua, ub = dev(u0), dev(u0)
    srj.srj_sweeps(c, ua, dev(f), 0, 57)
    d = srj.srj_plan((300, 200), 1.0 / 301, P=5)
    srj.srj_plan_set_fusion(d, 0)
    srj.srj_sweeps(d, ub, dev(f), 0, 57)
    assert np.array_equal(host(ua), host(ub))
    del wl
    with pytest.raises(srj.SrjError):
        srj.srj_plan_tune_cached(c, os.path.join(str(tmp_path), "no_such_dir", "x.txt"))
