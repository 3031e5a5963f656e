"""Benchmark: SRJ time-to-tolerance and GLUP/s on one MI355X.

Default workload: 2D Poisson, 4096 x 4096 interior points, 5-point stencil, Dirichlet ring
U(-1,1) (seed 0), f = 32 seeded Gaussian blobs, SRJ with a P = 10 schedule optimised for
the grid's exact smallest Jacobi symbol, binary64, stop at relative residual 1e-10.

One step = one complete solve from the same initial state (copy of u0, inputs resident
in HBM, the plan -- schedule and buffers -- built beforehand).  value = interior points x
sweeps / wall time per solve (GLUP/s).  The roofline object describes the dominant
kernel (the temporally blocked 2D sweep): its algorithmic HBM bytes per launch (read u
and b once, write u once: 24 B per interior point) over its average launch duration,
timed with HIP events on the plan's stream.  The CPU baseline is the oracle's plain C
loops timed on the host on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_PER_POINT_F64 = 24.0  # read u, read b, write u


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1511_04292_amd", "csrc", "sweep2d_tb.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}|{workload}")
    except (ValueError, OSError):
        return None
    if not rec or rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(wl, levels, sweeps_to_tol, seconds_target=15.0):
    """The oracle (plain C loops, OpenMP over rows) timed on the host: its own schedule for
    the same grid, a bounded number of sweeps of the full workload."""
    from oracle import _clib, sweeps
    from oracle import schedule as S

    km = S.kappa_min_dirichlet(wl["n"])
    o = S.optimal(levels, km)
    q = S.q_floor(o["beta"])
    seq_w = S.weight_sequence(o["w"], S.order_balanced(o["w"], q, km))
    b = sweeps.rhs(wl["f"], wl["h"])
    c = sweeps.coefficients(seq_w, len(wl["n"]))
    u = wl["u0"].copy()
    u = sweeps.run(u, b, c, 1)  # first touch
    t0 = time.perf_counter()
    u = sweeps.run(u, b, c, 3, k0=1)
    t1 = (time.perf_counter() - t0) / 3
    nsw = max(1, int(seconds_target / max(t1, 1e-6)))
    t0 = time.perf_counter()
    u = sweeps.run(u, b, c, nsw, k0=4)
    dt = time.perf_counter() - t0
    pts = math.prod(wl["n"])
    rate = pts * nsw / dt
    return {"value": round(rate / 1e9, 4), "unit": "GLUP/s", "cores": _clib.max_threads(),
            "kind": "oracle",
            "sample": f"{nsw} scheduled FP64 sweeps of the full {'x'.join(map(str, wl['n']))} grid "
                      f"({dt:.1f} s timed); time-to-tolerance extrapolated to {sweeps_to_tol} sweeps: "
                      f"{sweeps_to_tol * pts / rate:.0f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--levels", type=int, default=10)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--fuse", type=int, default=None, help="sweeps fused per launch (0 = unfused)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--workloads", default="all", choices=["all", "main"],
                    help="'all' also measures the 3D, batched and differentiable workloads")
    ap.add_argument("--kernel-only", action="store_true",
                    help="counter-collection run: one 1 GiB read / 1 GiB write calibration kernel, then "
                         "20 fused and 20 unfused sweep launches on the workload; prints no JSON")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the SRJ solver here runs on a single MI355X; "
              "multi-GPU runs are not part of this build.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1511_04292_amd import srj, workloads

    n = args.n
    t0 = time.perf_counter()
    wl = workloads.blobs_2d(n, seed=0)
    t_gen = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    u0 = torch.from_numpy(wl["u0"]).to(dev)
    f = torch.from_numpy(wl["f"]).to(dev)
    u = torch.empty_like(u0)

    t0 = time.perf_counter()
    plan = srj.srj_plan(wl["n"], wl["h"], P=args.levels)
    t_plan = time.perf_counter() - t0
    if args.fuse is not None:
        srj.srj_plan_set_fusion(plan, args.fuse)
    desc = srj.srj_plan_describe(plan)
    M = int(desc["M"])
    pts = n * n

    if args.kernel_only:
        big = torch.full((1 << 27,), 1.0, dtype=torch.float64, device=dev)  # 1 GiB
        big2 = torch.empty_like(big)
        torch.mul(big, 2.0, out=big2)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        fuse = int(desc["fused_sweeps"])
        u.copy_(u0)
        srj.srj_sweeps(plan, u, f, 0, 20 * fuse)
        srj.srj_plan_set_fusion(plan, 0)
        u.copy_(u0)
        srj.srj_sweeps(plan, u, f, 0, 20)
        torch.cuda.synchronize()
        if args.workloads == "all":
            del plan, u, u0, f
            w3 = workloads.smooth_3d(512, seed=0)
            u3 = torch.from_numpy(w3["u0"]).to(dev)
            f3 = torch.from_numpy(w3["f"]).to(dev)
            for fmt in ("f64", "f32"):
                p3 = srj.srj_plan(w3["n"], w3["h"], P=8, dtype=fmt)
                srj.srj_sweeps(p3, u3.clone(), f3, 0, 20)
                del p3
            torch.cuda.synchronize()
        print("kernel-only run done", flush=True)
        return

    def step():
        u.copy_(u0)
        return srj.srj_solve(plan, u, f, args.tol, 100 * M)

    for _ in range(args.warmup):
        info = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(step())
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    info = infos[-1]
    sweeps_done = int(info["sweeps"])
    glups = pts * sweeps_done / dt / 1e9

    # dominant kernel: average launch of the fused sweep over whole cycles' worth of launches
    fuse = int(desc["fused_sweeps"])
    nsw = min(M, 8 * 256) if fuse > 0 else min(M, 256)
    nsw -= nsw % max(fuse, 1)
    u.copy_(u0)
    srj.srj_sweeps(plan, u, f, 0, nsw)  # warm
    u.copy_(u0)
    sec, launches = srj.srj_sweeps(plan, u, f, 0, nsw)
    avg_launch = sec / launches
    bytes_launch = B_PER_POINT_F64 * pts
    achieved = bytes_launch / avg_launch / 1e9
    kname = f"k_sweep2d_tb<double,{fuse},2,3>" if fuse > 0 else "k_sweep2d<double>"
    wname = f"blobs2d_{n}x{n}_f64"
    traffic = measured_traffic(kname, wname)

    # unfused reference sweep on the same grid, for the per-sweep HBM figure
    srj.srj_plan_set_fusion(plan, 0)
    u.copy_(u0)
    srj.srj_sweeps(plan, u, f, 0, 64)
    u.copy_(u0)
    sec0, l0 = srj.srj_sweeps(plan, u, f, 0, 256)
    srj.srj_plan_set_fusion(plan, fuse)
    unfused_gbs = B_PER_POINT_F64 * pts / (sec0 / l0) / 1e9

    out = {
        "metric": "SRJ GLUP/s + time-to-1e-10 residual (4096^2 2D, 512^3 3D); % HBM roofline",
        "value": round(glups, 3),
        "unit": "GLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian-blob source, U(-1,1) Dirichlet ring)",
        "config": {"workload": f"2D Poisson {n}x{n} interior, 5-point, Dirichlet, SRJ P={args.levels} "
                               f"(M={M}), FP64, tol {args.tol:g}",
                   "n": n, "levels": args.levels, "M": M, "tol": args.tol, "fused_sweeps": fuse},
        "time_to_tol_s": round(dt, 4),
        "sweeps": sweeps_done,
        "cycles": int(info["cycles"]),
        "relres": info["relres"],
        "status": info["status"],
        "effective_per_sweep_hbm_frac": round(glups * B_PER_POINT_F64 / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kname, "avg_launch_us": round(avg_launch * 1e6, 2),
                     "sweeps_per_launch": fuse if fuse > 0 else 1,
                     "algorithmic_bytes_per_launch": bytes_launch},
        "unfused_sweep": {"kernel": "k_sweep2d<double>", "avg_launch_us": round(sec0 / l0 * 1e6, 2),
                          "achieved_GBs": round(unfused_gbs, 1),
                          "frac": round(unfused_gbs / HBM_PEAK_GBS, 4)},
        "schedule": {"omega1": desc["omega"][0], "rho": desc["rho"], "gamma_q_max": desc["gamma_q_max"],
                     "prefix_peak_log10": desc["prefix_peak_log10"]},
        "plan_seconds": round(t_plan, 3),
        "input_gen_seconds": round(t_gen, 2),
        "pcie_note": "inputs resident in HBM before timing; host<->device copies excluded",
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.levels, sweeps_done, args.cpu_seconds)
    if args.workloads == "all":
        del plan, u, u0, f
        torch.cuda.empty_cache()
        other = {}
        for name, fn in (("smooth3d_512", bench_3d), ("batch_1024", bench_batch), ("adjoint_2048", bench_adjoint)):
            print(f"bench: {name} ...", file=sys.stderr, flush=True)
            other[name] = fn(torch, srj, workloads)
            torch.cuda.empty_cache()
        out["other_workloads"] = other
    print(json.dumps(out), flush=True)


def bench_3d(torch, srj, workloads, n=512, levels=8, tol=1e-10):
    """512^3 Poisson, P = 8: FP64 SRJ, and FP64 refinement around FP32 and BF16-storage sweeps."""
    wl = workloads.smooth_3d(n, seed=0)
    u0 = torch.from_numpy(wl["u0"]).to("cuda:0")
    f = torch.from_numpy(wl["f"]).to("cuda:0")
    del wl
    pts = n ** 3
    res = {"workload": f"3D Poisson {n}^3 interior, 7-point, zero Dirichlet ring, f = U(-1,1) smoothed once, "
                       f"SRJ P={levels}, tol {tol:g}"}
    ref = None
    for fmt in ("f64", "f32", "bf16"):
        plan = srj.srj_plan((n, n, n), 1.0 / (n + 1), P=levels, dtype=fmt)
        u = u0.clone()
        sec, launches = srj.srj_sweeps(plan, u, f, 0, 32)
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = int(srj.srj_plan_describe(plan)["M"])
        if fmt == "f64":
            info = srj.srj_solve(plan, u, f, tol, 100 * M)
        else:
            info = srj.srj_solve_ir(plan, u, f, tol, 1, 100)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        bpp = {"f64": 24, "f32": 12, "bf16": 6}[fmt]
        r = {"time_to_tol_s": round(dt, 4), "sweeps": int(info["sweeps"]), "cycles_or_outer": int(info["cycles"]),
             "relres": info["relres"], "status": info["status"], "GLUP_s": round(pts * info["sweeps"] / dt / 1e9, 2),
             "sweep_kernel_us": round(sec / launches * 1e6, 1),
             "sweep_kernel_GBs": round(bpp * pts / (sec / launches) / 1e9, 1),
             "sweep_kernel_hbm_frac": round(bpp * pts / (sec / launches) / 1e9 / HBM_PEAK_GBS, 4)}
        if fmt == "f64":
            ref = u
            r["M"] = int(srj.srj_plan_describe(plan)["M"])
        else:
            r["max_abs_err_vs_f64_rel"] = float((u - ref).abs().max() / ref.abs().max())
            del u
        res[fmt if fmt == "f64" else f"{fmt}_refined"] = r
        del plan
    return res


def bench_batch(torch, srj, workloads, count=1024, tol=1e-10):
    """1024 independent 2D problems, N log-uniform in [32, 1024], P uniform in 3..8, binary32
    sweeps inside binary64 refinement, one batched device loop."""
    import numpy as np

    N, P = workloads.batch_sizes(count=count)
    probs, u0s, fs = [], [], []
    for j, (nn, pp) in enumerate(zip(N, P)):
        wl = workloads.batch_problem(int(nn), seed=10000 + j)
        probs.append(dict(n=(int(nn), int(nn)), h=wl["h"], P=int(pp)))
        u0s.append(torch.from_numpy(wl["u0"]).to("cuda:0"))
        fs.append(torch.from_numpy(wl["f"]).to("cuda:0"))
    t0 = time.perf_counter()
    b = srj.srj_batch_plan(probs, dtype="f32")
    t_plan = time.perf_counter() - t0
    us = [u.clone() for u in u0s]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, secs = srj.srj_batch_solve(b, us, fs, tol, 1, 2000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lup = sum(int(nn) * int(nn) * i["sweeps"] for nn, i in zip(N, infos))
    return {"workload": f"{count} 2D Poisson problems, N log-uniform [32, 1024], P in 3..8, f ~ N(0,1), "
                        f"FP32 sweeps in FP64 refinement, tol {tol:g}",
            "wall_s": round(dt, 3), "plan_s": round(t_plan, 2), "converged": sum(i["status"] == "ok" for i in infos),
            "total_points": int(sum(int(nn) ** 2 for nn in N)), "total_LUP": int(lup),
            "GLUP_s": round(lup / dt / 1e9, 2), "solves_per_s": round(count / dt, 2),
            "p50_problem_s": round(float(np.percentile(secs, 50)), 4),
            "p99_problem_s": round(float(np.percentile(secs, 99)), 4),
            "max_relres": max(i["relres"] for i in infos)}


def bench_adjoint(torch, srj, workloads, n=2048, levels=9, tol=1e-10):
    """Differentiable solve on 2048^2: forward SRJ and the adjoint SRJ backward."""
    from paper_1511_04292_amd.autograd import srj_solve_diff

    wl = workloads.adjoint_2d(n)
    f = torch.from_numpy(wl["f"]).to("cuda:0").requires_grad_(True)
    g = torch.from_numpy(wl["g"]).to("cuda:0").requires_grad_(True)
    ut = torch.from_numpy(wl["u_target"]).to("cuda:0")
    plan = srj.srj_plan((n, n), wl["h"], P=levels)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = srj_solve_diff(f, g, plan, tol=tol, tol_backward=1e-9)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = 0.5 * ((u - ut)[1:-1, 1:-1] ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return {"workload": f"2D {n}^2, f blobs and U(-1,1) ring as parameters, L = 1/2 ||u - u_target||^2, "
                        f"SRJ P={levels} forward to {tol:g}, adjoint to 1e-9 (binary64 floor of a smooth "
                        f"right-hand side is about 2e-10 here)",
            "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
            "loss": float(loss.detach())}


if __name__ == "__main__":
    main()
