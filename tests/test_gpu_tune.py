"""Autotuning of the launch shape: the tuner reports what it timed, changes only speed, and the
solves after it stay bit-identical to the oracle."""
import numpy as np
import pytest
import torch

from oracle import schedule as S
from oracle import sweeps
from paper_1511_04292_amd import srj, workloads

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def oracle_sched(n, P):
    km = S.kappa_min_dirichlet(n)
    o = S.optimal(P, km)
    q = S.q_floor(o["beta"])
    return o["w"], q, S.order_balanced(o["w"], q, km)


def case(n, seed):
    rng = np.random.default_rng(seed)
    full = tuple(x + 2 for x in reversed(n))
    u0 = workloads.random_ring(full, rng)
    f = np.zeros(full)
    f[tuple(slice(1, -1) for _ in n)] = rng.standard_normal(tuple(reversed(n)))
    return u0, f


@pytest.mark.parametrize("n,P", [((301, 222), 4), ((37, 29, 23), 3)])
def test_plan_tune_then_solve_bitwise(n, P):
    h = 1.0 / (max(n) + 1)
    w, q, seq = oracle_sched(n, P)
    plan = srj.srj_plan(n, h, omega=w, q=q, sequence=seq)
    before = srj.srj_plan_describe(plan)["fused_sweeps"]
    t = srj.srj_plan_tune(plan)
    assert t["candidates"] == (29 if len(n) == 2 else 7)
    assert 0 < t["us_per_sweep"] <= t["us_per_sweep_before"]
    assert srj.srj_plan_describe(plan)["fused_sweeps"] == t["fused_sweeps"]
    assert before == 10 if len(n) == 2 else before in (3, 4, 5)  # 3D: from the launch-shape model
    u0, f = case(n, 21)
    u = torch.from_numpy(u0).to(DEV)
    info = srj.srj_solve(plan, u, torch.from_numpy(f).to(DEV), 1e-10, 10 ** 5)
    ref = sweeps.solve(u0, f, h, np.asarray(w)[seq], 1e-10, 10 ** 5)
    torch.cuda.synchronize()
    assert info["status"] == "ok" and info["sweeps"] == ref["sweeps"]
    assert np.array_equal(u.cpu().numpy(), ref["u"])


def test_batch_tune_then_solve_bitwise():
    sizes = [(40, 40), (130, 97), (257, 200), (64, 65), (9, 300)]
    levels = [3, 4, 5, 3, 4]
    probs, data, refs = [], [], []
    for i, (n, P) in enumerate(zip(sizes, levels)):
        w, q, seq = oracle_sched(n, P)
        h = 1.0 / (max(n) + 1)
        u0, f = case(n, 40 + i)
        probs.append(dict(n=n, h=h, omega=w, q=q, sequence=seq))
        data.append((u0, f))
        refs.append(sweeps.solve_ir(u0, f, h, np.asarray(w)[seq], 1e-10, 1, 400, "f32"))
    b = srj.srj_batch_plan(probs, dtype="f32")
    t = srj.srj_batch_tune(b)
    assert t["fused_sweeps"] == 10 and t["seg_rows"] in (32, 64, 128, 256) and t["candidates"] >= 4
    assert 0 < t["us_per_sweep"] <= t["us_per_sweep_before"]
    for rep in range(2):  # the tuned batch solves, twice, from the same inputs
        us = [torch.from_numpy(u0).to(DEV) for u0, _ in data]
        fs = [torch.from_numpy(f).to(DEV) for _, f in data]
        infos, _ = srj.srj_batch_solve(b, us, fs, 1e-10, 1, 400)
        torch.cuda.synchronize()
        for i, (info, ref) in enumerate(zip(infos, refs)):
            assert info["status"] == "ok" and info["cycles"] == ref["outer"], (rep, i, info, ref["outer"])
            assert np.array_equal(us[i].cpu().numpy(), ref["u"]), (rep, i)
