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
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
B_PER_POINT_F64 = 24.0  # read u, read b, write u


# Sources the fused 2D sweep is compiled from: counter-derived traffic is used only while
# they are unchanged.
FUSED_SOURCES = ("sweep2d_tb.hip", "tb_core.h", "formats.h")


OTHER_NAMES = ("small_2d_64", "case_study_585x280", "neumann_calibration_256", "planner_variants",
               "grad_shafranov_300", "spherical_poisson_512", "smooth3d_512", "batch_1024", "adjoint_2048",
               "huge_2d_32768")


def other_workloads():
    """The other configurations measured in the same run, in the order they run."""
    fns = (bench_small_2d, bench_case_study, bench_neumann_calibration, bench_planner_variants,
           bench_grad_shafranov, bench_spherical_poisson, bench_3d, bench_batch, bench_adjoint, bench_huge_2d)
    return list(zip(OTHER_NAMES, fns))


def kernel_source_hash():
    """Hash of the fused kernel's code: its sources with comments, indentation and blank lines
    removed, so that editing a comment leaves counters taken on the same code valid."""
    h = hashlib.sha256()
    for name in FUSED_SOURCES:
        with open(os.path.join(ROOT, "paper_1511_04292_amd", "csrc", name)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].strip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def ingest_counters(fetch_dir, write_dir, workload="blobs2d_4096x4096_f64"):
    """Turn the counter CSVs of two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
    `bench.py --kernel-only` into HBM bytes per launch: each counter is scaled by what it reads
    for the calibration kernel (torch's elementwise multiply over 1 GiB in, 1 GiB out).  Writes
    profiles/traffic.json and returns a markdown table."""
    import csv
    import glob

    def per_kernel(d, counter):
        acc = {}
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                if r["Counter_Name"] != counter:
                    continue
                k = r["Kernel_Name"]
                acc.setdefault(k, []).append(float(r["Counter_Value"]))
        return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}

    fetch = per_kernel(fetch_dir, "FETCH_SIZE")
    write = per_kernel(write_dir, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    cal = [k for k in fetch if "elementwise" in k and "Mul" in k]
    if not cal:
        raise SystemExit("no calibration kernel in the counter runs")
    fscale = gib_kib / fetch[cal[0]][0]
    wscale = gib_kib / write[cal[0]][0]
    n = 4096
    rows, out = [], {}
    for k, (fk, cnt) in sorted(fetch.items()):
        if "srj::" not in k:
            continue
        wk = write.get(k, (float("nan"), 0))[0]
        rb = fk * 1024 * fscale
        wb = wk * 1024 * wscale
        short = k.split("(")[0].replace("void ", "").replace("srj::", "")
        rows.append(f"| `{short}` | {cnt} | {fk:.0f} | {wk:.0f} | {rb / 1e6:.1f} + {wb / 1e6:.1f} = {(rb + wb) / 1e6:.1f} |")
        if short.startswith("k_sweep2d_tb<double,"):
            key = short.replace(" ", "")
            out[f"{key}|{workload}"] = {
                "bytes_per_launch": int(rb + wb), "read_bytes": int(rb), "write_bytes": int(wb),
                "fetch_scale": round(fscale, 4), "write_scale": round(wscale, 4),
                "kernel_source_sha256_16": kernel_source_hash(),
                "kernel_sources": [f"paper_1511_04292_amd/csrc/{x}" for x in FUSED_SOURCES],
                "algorithmic_bytes_per_launch": 24 * n * n}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    head = (f"Calibration: FETCH_SIZE scale {fscale:.4f}, WRITE_SIZE scale {wscale:.4f} "
            f"(torch multiply over 1 GiB binary64 in, 1 GiB out)\n\n"
            "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled HBM MB (read + write) |\n"
            "|---|---|---|---|---|")
    return head + "\n" + "\n".join(rows)


def summarize_trace(trace_dir):
    """Per-kernel launch statistics from a `rocprofv3 --kernel-trace` CSV, split by grid size
    (so launches of the same kernel on different workloads stay apart), as a markdown table."""
    import csv
    import glob

    groups = {}
    for fn in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "")
            key = (name.split("(")[0].replace("void ", ""),
                   f'{r["Grid_Size_X"]}x{r["Grid_Size_Y"]}x{r["Grid_Size_Z"]}')
            groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in groups.values())
    timeline = batch_timeline(trace_dir)
    lines = ["| kernel | grid (threads) | calls | total ms | average us | min us | max us | % |",
             "|---|---|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) < 1e-3 * total:
            continue
        lines.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / 1e3:.2f} | {sum(v) / len(v):.2f} | "
                     f"{min(v):.1f} | {max(v):.1f} | {100 * sum(v) / total:.2f} |")
    if timeline:
        lines += ["", timeline]
    return "\n".join(lines)


def batch_timeline(trace_dir):
    """The batched solve's launches over time (the last run of k_batch_step launches without a
    gap above 5 ms, i.e. the solve and not the tuner): how long launches take as problems
    finish, and how much of the wall the gaps between launches are."""
    import csv
    import glob

    ev = []
    for fn in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(fn)):
            if "k_batch_step" in r["Kernel_Name"]:
                ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    if not ev:
        return ""
    ev.sort()
    i0 = 0
    for i in range(1, len(ev)):
        if ev[i][0] - ev[i - 1][1] > 5_000_000:
            i0 = i
    ev = ev[i0:]
    t0 = ev[0][0]
    span = (ev[-1][1] - t0) / 1e9
    busy = sum(e - s for s, e in ev) / 1e9
    out = [f"Batched solve: {len(ev)} launches in {span:.3f} s, {busy:.3f} s inside launches, "
           f"{span - busy:.3f} s between them.", "",
           "| from s | launches | mean launch us | share of the interval inside launches |", "|---|---|---|---|"]
    step = 0.25
    t = 0.0
    while t < span:
        sel = [(s, e) for s, e in ev if t <= (s - t0) / 1e9 < t + step]
        if sel:
            d = sum(e - s for s, e in sel) / len(sel) / 1e3
            out.append(f"| {t:.2f} | {len(sel)} | {d:.1f} | {sum(e - s for s, e in sel) / 1e9 / step:.2f} |")
        t += step
    return "\n".join(out)


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


def cpu_baseline(wl, levels, sweeps_to_tol, seconds_target=15.0, single_seconds=5.0):
    """The oracle (plain C loops, OpenMP over rows) timed on the host: its own schedule for
    the same grid, a bounded number of sweeps of the full workload, on all threads and on one
    thread; and the 64^2 case (SRJ P = 2 and plain Jacobi) run to full convergence."""
    from oracle import _clib, sweeps
    from oracle import schedule as S

    km = S.kappa_min_dirichlet(wl["n"])
    o = S.optimal(levels, km)
    q = S.q_floor(o["beta"])
    seq_w = S.weight_sequence(o["w"], S.order_balanced(o["w"], q, km))
    b = sweeps.rhs(wl["f"], wl["h"])
    c = sweeps.coefficients(seq_w, len(wl["n"]))
    pts = math.prod(wl["n"])

    def timed(target):
        u = wl["u0"].copy()
        u = sweeps.run(u, b, c, 1)  # first touch
        t0 = time.perf_counter()
        u = sweeps.run(u, b, c, 3, k0=1)
        t1 = (time.perf_counter() - t0) / 3
        nsw = max(1, int(target / max(t1, 1e-6)))
        t0 = time.perf_counter()
        sweeps.run(u, b, c, nsw, k0=4)
        return nsw, time.perf_counter() - t0

    threads = _clib.max_threads()
    nsw, dt = timed(seconds_target)
    rate = pts * nsw / dt
    prev = _clib.set_threads(1)
    try:
        nsw1, dt1 = timed(single_seconds)
    finally:
        _clib.set_threads(prev)
    rate1 = pts * nsw1 / dt1
    out = {"value": round(rate / 1e9, 4), "unit": "GLUP/s", "cores": threads, "kind": "oracle",
           "sample": f"{nsw} scheduled FP64 sweeps of the full {'x'.join(map(str, wl['n']))} grid "
                     f"({dt:.1f} s timed, {threads} threads); time-to-tolerance extrapolated to "
                     f"{sweeps_to_tol} sweeps: {sweeps_to_tol * pts / rate:.0f} s",
           "single_thread": {"value": round(rate1 / 1e9, 4), "unit": "GLUP/s", "cores": 1,
                             "sample": f"{nsw1} sweeps of the same grid ({dt1:.1f} s timed); "
                                       f"time-to-tolerance extrapolated: {sweeps_to_tol * pts / rate1:.0f} s"}}
    # 64^2: SRJ P = 2 (the oracle's schedule for the grid) and Jacobi to relres 1e-10
    from paper_1511_04292_amd import workloads

    w1 = workloads.small_2d(64, seed=0)
    km1 = S.kappa_min_dirichlet(w1["n"])
    o1 = S.optimal(2, km1)
    q1 = S.q_floor(o1["beta"])
    wseq1 = S.weight_sequence(o1["w"], S.order_balanced(o1["w"], q1, km1))
    small = {}
    for name, ws in (("srj_P2", wseq1), ("jacobi", [1.0])):
        t0 = time.perf_counter()
        r = sweeps.solve(w1["u0"], w1["f"], w1["h"], ws, 1e-10, 10 ** 7)
        small[name] = {"seconds": round(time.perf_counter() - t0, 3), "sweeps": int(r["sweeps"]),
                       "relres": r["relres"], "status": r["status"]}
    small["measured_acceleration"] = round(small["jacobi"]["sweeps"] / max(1, small["srj_P2"]["sweeps"]), 3)
    out["small_2d_64"] = small
    return out


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
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="read the counter CSVs of two --kernel-only runs under rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE, write profiles/traffic.json, print a table")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="print per-kernel, per-grid launch statistics of a rocprofv3 --kernel-trace run")
    ap.add_argument("--only", choices=OTHER_NAMES, default=None,
                    help="run one of the other workloads alone and print its JSON (profiling aid)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="counter-collection run: one 1 GiB read / 1 GiB write calibration kernel, then "
                         "20 fused and 20 unfused sweep launches on the workload, 20 fused launches in "
                         "binary32 and bfloat16, and 20 sweeps of the 512^3 grid in each format; prints "
                         "no JSON")
    args = ap.parse_args()
    if args.ingest_counters:
        print(ingest_counters(*args.ingest_counters))
        return
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the SRJ solver runs on a single MI355X and has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1511_04292_amd import srj, workloads

    if args.only:
        fn = dict(other_workloads())[args.only]
        print(f"bench: {args.only} ...", file=sys.stderr, flush=True)
        print(json.dumps({"workload": args.only, "result": fn(torch, srj, workloads)}))
        return

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
    if args.fuse is not None or args.kernel_only:
        # counter runs measure the default launch shape only
        if args.fuse is not None:
            srj.srj_plan_set_fusion(plan, args.fuse)
        tuned = {"fused_sweeps": int(srj.srj_plan_describe(plan)["fused_sweeps"]), "seg_rows": 0, "tuned": False}
    else:
        t0 = time.perf_counter()
        tuned = dict(srj.srj_plan_tune(plan), tuned=True, seconds=round(time.perf_counter() - t0, 3))
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
            # the binary32 and bfloat16 fused 2D sweeps on the same grid (their default depth)
            for fmt in ("f32", "bf16"):
                pl = srj.srj_plan(wl["n"], wl["h"], P=args.levels, dtype=fmt)
                fl = int(srj.srj_plan_describe(pl)["fused_sweeps"])
                u.copy_(u0)
                srj.srj_sweeps(pl, u, f, 0, 20 * fl)
                del pl
            torch.cuda.synchronize()
            del plan, u, u0, f
            w3 = workloads.smooth_3d(512, seed=0)
            u3 = torch.from_numpy(w3["u0"]).to(dev)
            f3 = torch.from_numpy(w3["f"]).to(dev)
            for fmt in ("f64", "f32", "bf16"):
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
    hint = 2 if int(desc.get("store_nt", 0)) else 0  # the kernel's store-hint template argument
    kname = f"k_sweep2d_tb<double,{fuse},2,3,{hint}>" if fuse > 0 else "k_sweep2d<double>"
    wname = f"blobs2d_{n}x{n}_f64"
    # counters were taken on the default launch shape (the default depth, segment height
    # from the occupancy); the record is keyed by kernel (and so depth), another segment
    # height has no committed traffic
    traffic = measured_traffic(kname, wname) if int(tuned["seg_rows"]) == 0 else None

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
                   "n": n, "levels": args.levels, "M": M, "tol": args.tol, "fused_sweeps": fuse,
                   "seg_rows": int(tuned["seg_rows"])},
        "launch_tuning": tuned,
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
        for name, fn in other_workloads():
            print(f"bench: {name} ...", file=sys.stderr, flush=True)
            other[name] = fn(torch, srj, workloads)
            torch.cuda.empty_cache()
        out["other_workloads"] = other
    print(json.dumps(out), flush=True)


def exact_dirichlet(u_ring, f, h):
    """Exact solution of the discrete Dirichlet problem A u = h^2 f + (ring terms): the
    5-/7-point Laplacian is diagonalised by the type-I DST along every axis, with eigenvalues
    sum_i 4 sin^2(k_i pi / (2 (n_i + 1))).  Host binary64 (scipy), all threads."""
    import numpy as np
    import scipy.fft

    nd = f.ndim
    inner = tuple(slice(1, -1) for _ in range(nd))
    rhs = (float(h) * float(h)) * f[inner]
    g = np.array(u_ring, copy=True)
    g[inner] = 0.0
    for ax in range(nd):
        lo = [slice(1, -1)] * nd
        hi = [slice(1, -1)] * nd
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        rhs = rhs + g[tuple(lo)] + g[tuple(hi)]
    lam = np.zeros(rhs.shape)
    for ax, m in enumerate(rhs.shape):
        k = np.arange(1, m + 1, dtype=np.float64)
        shp = [1] * nd
        shp[ax] = m
        lam = lam + (4.0 * np.sin(k * np.pi / (2.0 * (m + 1))) ** 2).reshape(shp)
    t = scipy.fft.dstn(rhs, type=1, norm="ortho", workers=-1)
    del rhs
    t /= lam
    del lam
    u = np.array(u_ring, copy=True)
    u[inner] = scipy.fft.dstn(t, type=1, norm="ortho", workers=-1)
    return u


def bench_3d(torch, srj, workloads, n=512, levels=8, tol=1e-10):
    """512^3 Poisson, P = 8: FP64 SRJ, and FP64 refinement around FP32 and BF16-storage sweeps.
    Each result is compared with the exact discrete solution (DST-I, host binary64)."""
    import numpy as np

    wl = workloads.smooth_3d(n, seed=0)
    u0 = torch.from_numpy(wl["u0"]).to("cuda:0")
    f = torch.from_numpy(wl["f"]).to("cuda:0")
    t0 = time.perf_counter()
    ustar = exact_dirichlet(wl["u0"], wl["f"], wl["h"])
    t_exact = time.perf_counter() - t0
    ustar_max = float(np.max(np.abs(ustar)))
    del wl
    pts = n ** 3
    res = {"workload": f"3D Poisson {n}^3 interior, 7-point, zero Dirichlet ring, f = U(-1,1) smoothed once, "
                       f"SRJ P={levels}, tol {tol:g}"}
    ref = None
    for fmt in ("f64", "f32", "bf16"):
        plan = srj.srj_plan((n, n, n), 1.0 / (n + 1), P=levels, dtype=fmt)
        tuned = srj.srj_plan_tune(plan)
        # launch timing over a whole number of launches at the chosen depth: 8 untimed, then 24
        fz = max(1, int(srj.srj_plan_describe(plan)["fused_sweeps"]))
        nsw = 24 * fz
        u = u0.clone()
        srj.srj_sweeps(plan, u, f, 0, 8 * fz)
        sec, launches = srj.srj_sweeps(plan, u, f, 8 * fz, nsw)
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
        launch_s = sec / launches
        per_sweep = sec / nsw
        r = {"time_to_tol_s": round(dt, 4), "sweeps": int(info["sweeps"]), "cycles_or_outer": int(info["cycles"]),
             "relres": info["relres"], "status": info["status"], "GLUP_s": round(pts * info["sweeps"] / dt / 1e9, 2),
             "fused_sweeps": int(srj.srj_plan_describe(plan)["fused_sweeps"]),
             "launch_tuning": tuned,
             "launch_us": round(launch_s * 1e6, 1), "per_sweep_us": round(per_sweep * 1e6, 1),
             # algorithmic bytes of one launch (u, b read once, u written once) over its time
             "launch_algorithmic_GBs": round(bpp * pts / launch_s / 1e9, 1),
             # effective sweep rate over the unfused sweep's HBM roofline (8 TB/s / bytes per update)
             "per_sweep_hbm_roofline_frac": round(pts / per_sweep / (HBM_PEAK_GBS * 1e9 / bpp), 3)}
        # max |u - u*| / max |u*| against the exact discrete solution
        r["err_vs_exact"] = float(np.max(np.abs(u.cpu().numpy() - ustar))) / ustar_max
        if fmt == "f64":
            ref = u
            r["M"] = int(srj.srj_plan_describe(plan)["M"])
        else:
            r["max_abs_err_vs_f64_gpu_rel"] = float((u - ref).abs().max() / ref.abs().max())
            del u
        res[fmt if fmt == "f64" else f"{fmt}_refined"] = r
        del plan
    res["exact_reference"] = (f"u* from the type-I DST of the discrete problem on the host "
                              f"({t_exact:.1f} s); err_vs_exact = max|u - u*| / max|u*|")
    return res


def bench_small_2d(torch, srj, workloads, n=64, tol=1e-10):
    """64^2 Poisson (manufactured sin-sin source plus N(0, 1e-3^2) noise, zero ring): SRJ with
    the P = 2 schedule the product planner builds for the grid, against plain Jacobi (one
    weight 1, checked after every sweep), both to relres 1e-10 on the GPU.  The measured
    acceleration (Jacobi sweeps / SRJ sweeps) is reported beside the schedule's rho (Eq. rho)
    and the rate ratio log(Gamma_q) / log(1 - kappa_min) of the slowest mode."""
    wl = workloads.small_2d(n, seed=0)
    u0 = torch.from_numpy(wl["u0"]).to("cuda:0")
    f = torch.from_numpy(wl["f"]).to("cuda:0")
    out = {"workload": f"2D Poisson {n}x{n}, zero ring, f = 2 pi^2 sin sin + N(0, 1e-3^2), tol {tol:g}"}
    plans = {"srj_P2": srj.srj_plan(wl["n"], wl["h"], P=2),
             "jacobi": srj.srj_plan(wl["n"], wl["h"], omega=[1.0], q=[1])}
    for name, plan in plans.items():
        d = srj.srj_plan_describe(plan)
        u = u0.clone()
        srj.srj_solve(plan, u, f, tol, 10 ** 7)  # warm
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = srj.srj_solve(plan, u, f, tol, 10 ** 7)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": round(dt, 5), "sweeps": int(info["sweeps"]), "relres": info["relres"],
                     "status": info["status"], "device_seconds": round(info["seconds"], 5),
                     "omega": [float(x) for x in d["omega"]], "q": [int(x) for x in d["q"]], "M": int(d["M"])}
        if name == "srj_P2":
            out[name]["rho"] = d["rho"]
            out[name]["gamma_q_max"] = d["gamma_q_max"]
            km = d["kappa_min"]
    out["measured_acceleration"] = round(out["jacobi"]["sweeps"] / max(1, out["srj_P2"]["sweeps"]), 3)
    out["predicted_acceleration_slowest_mode"] = round(
        math.log(out["srj_P2"]["gamma_q_max"]) / math.log(1.0 - km), 3)
    out["time_ratio_jacobi_over_srj"] = round(out["jacobi"]["seconds"] / out["srj_P2"]["seconds"], 3)
    return out


def bench_case_study(torch, srj, workloads, tol=1e-10):
    """The Dirichlet case study of Sec. 5.1: -lap u = (x^2 + y^2) e^(xy) on the unit square cut
    into 585 x 280 zones (584 x 279 interior points, h = (1/585, 1/280)), u = -e^(xy) on the
    boundary.  SRJ P = 10 with the Neumann table rows the paper uses (N = 550, and N = 250
    from N_eff = 252.56 of Eq. effectiveNDirichlet), with the schedule for this grid's own
    smallest Jacobi symbol, and plain Jacobi; all to relres 1e-10 (checked at cycle ends,
    every sweep for Jacobi), binary64, one sweep per launch (unequal spacings)."""
    import numpy as np

    wl = workloads.exp_xy_unit_square(585, 280)
    u0 = torch.from_numpy(wl["u0"]).to("cuda:0")
    f = torch.from_numpy(wl["f"]).to("cuda:0")
    out = {"workload": "Sec. 5.1 case study: unit square, 585 x 280 zones, f = (x^2+y^2) e^(xy), "
                       "u = -e^(xy) on the boundary, P = 10, tol 1e-10"}
    plans = {"srj_N550": dict(P=10, n_eff=550.0), "srj_N250": dict(P=10, n_eff=250.0),
             "srj_exact_kappa_min": dict(P=10), "jacobi": dict(omega=[1.0], q=[1])}
    for name, kw in plans.items():
        plan = srj.srj_plan(wl["n"], wl["h"], **kw)
        d = srj.srj_plan_describe(plan)
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = srj.srj_solve(plan, u, f, tol, 10 ** 7)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        r = {"seconds": round(dt, 4), "sweeps": int(info["sweeps"]), "relres": info["relres"],
             "status": info["status"], "M": int(d["M"]),
             "max_err_vs_minus_exp_xy": float(np.max(np.abs(u.cpu().numpy() - wl["u_exact"])))}
        if name != "jacobi":
            r.update(q=[int(x) for x in d["q"]], omega_head=[float(x) for x in d["omega"][:3]],
                     rho_real=float(np.sum(d["omega"] * d["beta"])), rho_integer=d["rho"],
                     kappa_min=d["kappa_min"])
        out[name] = r
        del plan
    for name in ("srj_N550", "srj_N250", "srj_exact_kappa_min"):
        out[name]["measured_acceleration_vs_jacobi"] = round(out["jacobi"]["sweeps"] / out[name]["sweeps"], 2)
    out["N250_fewer_sweeps_than_N550_pct"] = round(
        100.0 * (1.0 - out["srj_N250"]["sweeps"] / out["srj_N550"]["sweeps"]), 2)
    return out


def bench_neumann_calibration(torch, srj, workloads, n=256, tol=1e-10):
    """The calibration of Sec. 4.1 on the paper's own model problem (Eq. Laplace: homogeneous
    Neumann, 256^2 cells, as in Fig. 2): SRJ P = 2..5 with the Neumann table rows for N = 256
    against plain Jacobi, from a seeded random start (U(-1,1)), to ||r|| <= 1e-10 ||r_0||
    (checked at cycle ends, every sweep for Jacobi).  Measured acceleration (Jacobi sweeps /
    SRJ sweeps) beside rho (Eq. rho) and the asymptotic rate ratio of the slowest mode."""
    import numpy as np

    rng = np.random.default_rng(0)
    u0h = rng.uniform(-1.0, 1.0, (n + 2, n + 2))
    u0 = torch.from_numpy(u0h).to("cuda:0")
    f = torch.zeros_like(u0)
    out = {"workload": f"Eq. Laplace, homogeneous Neumann, {n}^2 cells, random start U(-1,1), "
                       f"relres {tol:g} against the initial residual"}
    runs = {"jacobi": dict(omega=[1.0], q=[1])}
    for P in (2, 3, 4, 5):
        runs[f"srj_P{P}"] = dict(P=P, n_eff=float(n))
    for name, kw in runs.items():
        plan = srj.srj_plan((n, n), 1.0 / n, bc="neumann", **kw)
        d = srj.srj_plan_describe(plan)
        u = u0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = srj.srj_solve(plan, u, f, tol, 10 ** 8)
        torch.cuda.synchronize()
        r = {"seconds": round(time.perf_counter() - t0, 4), "sweeps": int(info["sweeps"]),
             "relres": info["relres"], "status": info["status"], "M": int(d["M"])}
        if name != "jacobi":
            km = d["kappa_min"]
            r.update(rho=round(float(np.sum(d["omega"] * d["beta"])), 3), q=[int(x) for x in d["q"]],
                     rate_ratio_slowest_mode=round(math.log(d["gamma_q_max"]) / math.log(1.0 - km), 3))
        out[name] = r
        del plan
    for P in (2, 3, 4, 5):
        out[f"srj_P{P}"]["measured_acceleration"] = round(out["jacobi"]["sweeps"] / out[f"srj_P{P}"]["sweeps"], 3)
    return out


def bench_planner_variants(torch, srj, workloads, tol=1e-10):
    """The planner variants of Sec. 4.3 measured on the device.
    (1) Integer conversions of beta / beta_1 in Fig. 4's setting: P = 6 for N = 256 on the
    Neumann model problem (Eq. Laplace, 256^2 cells, random start U(-1,1)), solved to relres
    1e-10: sweeps, and the cycle factor's maximum over the grid's symbols, per conversion
    (floor, nearest, ceiling, best per level); a conversion whose factor reaches 1 is refused.
    (2) The two step orders' rounding floors: binary32 and bfloat16 storage (plain SRJ, no
    refinement), 255^2 Dirichlet, zero ring, f ~ N(0,1), P = 8: the lowest relres of 40
    cycles' checks for the balanced and the even order."""
    import numpy as np

    out = {"workload": "Sec. 4.3 variants: q conversions at P = 6, N = 256 (Neumann, 256^2 cells, "
                       "relres 1e-10); balanced / even step orders' floors in binary32 / bfloat16 "
                       "(255^2 Dirichlet, P = 8, 40 cycles)"}
    n = 256
    rng = np.random.default_rng(0)
    u0 = torch.from_numpy(rng.uniform(-1.0, 1.0, (n + 2, n + 2))).to("cuda:0")
    f = torch.zeros_like(u0)
    conv = {}
    for mode, name in ((0, "floor"), (1, "nearest"), (2, "ceiling"), (3, "best")):
        try:
            plan = srj.srj_plan((n, n), 1.0 / n, P=6, n_eff=float(n), bc="neumann", q_rounding=mode)
        except srj.SrjError as e:
            conv[name] = {"refused": str(e)}
            continue
        d = srj.srj_plan_describe(plan)
        u = u0.clone()
        info = srj.srj_solve(plan, u, f, tol, 10 ** 7)
        conv[name] = {"q": [int(x) for x in d["q"]], "M": int(d["M"]), "sweeps": int(info["sweeps"]),
                      "status": info["status"], "gamma_q_max": d["gamma_q_max"],
                      "seconds": round(info["seconds"], 4)}
        del plan
    out["q_conversion_P6_N256"] = conv
    m = 255
    wl = workloads.batch_problem(m, seed=7)
    u0 = torch.from_numpy(wl["u0"]).to("cuda:0")
    f = torch.from_numpy(wl["f"]).to("cuda:0")
    floors = {}
    for fmt in ("f32", "bf16"):
        for ordering, oname in ((0, "balanced"), (1, "even")):
            plan = srj.srj_plan(wl["n"], wl["h"], P=8, dtype=fmt, ordering=ordering)
            M = int(srj.srj_plan_describe(plan)["M"])
            u = u0.clone()
            info = srj.srj_solve_ex(plan, u, f, 0.0, 40 * M, history_cap=64)
            h = [x for x in info["history"] if x == x]
            floors[f"{fmt}_{oname}"] = {"floor_relres": min(h) if h else None, "final_relres": info["relres"],
                                        "status": info["status"], "checks": info["checks"]}
            del plan
    out["order_floors_P8_255"] = floors
    return out


def bench_spherical_poisson(torch, srj, workloads, N=512, tol=1e-10):
    """Sec. 5.2: the Poisson equation in spherical coordinates, axisymmetric, multiplied by r^2
    (a variable-coefficient operator given point by point), N x N cells, solved with the
    Neumann-row schemes for N at P = 6 and P = 15 (the paper's smallest and largest) to relres
    1e-10, from a zero start (ab initio) and from the exact solution with 1/N relative noise
    (the paper's realistic calculation); error against the series solution."""
    import numpy as np

    out = {"workload": f"Sec. 5.2 spherical Poisson, axisymmetric, {N} x {N} cells, r^2-scaled operator, "
                       f"Neumann-row schemes for N = {N}, relres {tol:g}"}
    inner = (slice(1, -1), slice(1, -1))
    for start in ("zero", "realistic"):
        wl = workloads.spherical_poisson_2d(N, start=start, seed=0)
        coef = torch.from_numpy(wl["coef"]).to("cuda:0")
        f = torch.from_numpy(wl["f"]).to("cuda:0")
        for P in (6, 15):
            plan = srj.srj_plan_operator(wl["n"], coef, None, P=P, n_eff=float(N))
            d = srj.srj_plan_describe(plan)
            u = torch.from_numpy(wl["u0"]).to("cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = srj.srj_solve(plan, u, f, tol, 10 ** 7)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            err = float(np.max(np.abs(u.cpu().numpy() - wl["u_exact"])[inner]))
            out[f"{start}_P{P}"] = {"sweeps": int(info["sweeps"]), "seconds": round(dt, 4), "M": int(d["M"]),
                                    "relres": info["relres"], "status": info["status"],
                                    "fused_sweeps": int(d["fused_sweeps"]), "max_err_vs_series": err}
            del plan
    return out


def bench_grad_shafranov(torch, srj, workloads, n=298, tol=1e-12):
    """Sec. 5.3: the linear Grad-Shafranov equation on the paper's 300 x 300 points, test A
    (dipole boundary data) and test B (masked region), for several C, solved with the P = 14,
    N = 300 scheme to relres 1e-12 (the Jacobi-scaled residual, cycle ends), binary64, one
    sweep per launch.  The paper's Table 4 iteration counts are quoted as context (its own
    residual and stopping rule)."""
    import numpy as np

    table4 = {("A", 0.0): 5350, ("A", 0.2): 4660, ("A", 0.34): 49080, ("B", 0.0): 3450, ("B", 1.0): 3550,
              ("B", 1.47): 11620}
    out = {"workload": "Sec. 5.3 Grad-Shafranov, 300 x 300 points, P = 14 / N = 300 scheme, relres 1e-12"}
    for (test, C), printed in table4.items():
        wl = workloads.grad_shafranov(n, C, test)
        coef = torch.from_numpy(wl["coef"]).to("cuda:0")
        mask = torch.from_numpy(wl["mask"]).to("cuda:0") if wl["mask"] is not None else None
        plan = srj.srj_plan_operator(wl["n"], coef, mask, P=14, n_eff=300)
        u = torch.from_numpy(wl["u0"]).to("cuda:0")
        f = torch.from_numpy(wl["f"]).to("cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = srj.srj_solve(plan, u, f, tol, 10 ** 6)
        torch.cuda.synchronize()
        r = {"sweeps": int(info["sweeps"]), "seconds": round(time.perf_counter() - t0, 4), "relres": info["relres"],
             "status": info["status"], "paper_iterations": printed}
        if "u_exact" in wl:
            r["max_err_vs_dipole"] = float(np.max(np.abs(u.cpu().numpy() - wl["u_exact"])))
        out[f"test{test}_C{C}"] = r
        del plan, coef, mask
    return out


def bench_huge_2d(torch, srj, workloads, n=32768, levels=10, nsweeps=1000):
    """Throughput at 2^15 points per axis: 32768^2 binary64 (8.6 GB per field), the P = 10
    schedule for the grid, a fixed window of scheduled sweeps from the start of a cycle
    (2 full cycles would take minutes; the rate per sweep does not depend on the position in
    the cycle).  Inputs drawn on the device (workloads.blobs_2d_device)."""
    wl = workloads.blobs_2d_device(n, seed=0, device="cuda:0")
    u0, f = wl["u0"], wl["f"]
    t0 = time.perf_counter()
    plan = srj.srj_plan(wl["n"], wl["h"], P=levels)
    t_plan = time.perf_counter() - t0
    d = srj.srj_plan_describe(plan)
    fuse = int(d["fused_sweeps"])
    u = u0.clone()
    srj.srj_sweeps(plan, u, f, 0, 10 * fuse)  # warm
    u.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sec, launches = srj.srj_sweeps(plan, u, f, 0, nsweeps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pts = n * n
    launch_s = sec / launches
    return {"workload": f"2D Poisson {n}x{n}, Dirichlet ring U(-1,1), 32 Gaussian blobs, SRJ P={levels} "
                        f"(M={int(d['M'])}), binary64, {nsweeps} sweeps timed",
            "GLUP_s": round(pts * nsweeps / sec / 1e9, 1), "device_seconds": round(sec, 4),
            "wall_seconds_incl_copies": round(wall, 4), "launches": int(launches), "fused_sweeps": fuse,
            "launch_us": round(launch_s * 1e6, 1),
            "launch_algorithmic_GBs": round(B_PER_POINT_F64 * pts / launch_s / 1e9, 1),
            "launch_hbm_frac": round(B_PER_POINT_F64 * pts / launch_s / 1e9 / HBM_PEAK_GBS, 4),
            "M": int(d["M"]), "two_cycles_estimate_s": round(2 * int(d["M"]) * sec / nsweeps, 1),
            "plan_seconds": round(t_plan, 2)}


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
    tuned = srj.srj_batch_tune(b)
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
            "wall_s": round(dt, 3), "plan_s": round(t_plan, 2), "launch_tuning": tuned, "converged": sum(i["status"] == "ok" for i in infos),
            "total_points": int(sum(int(nn) ** 2 for nn in N)), "total_LUP": int(lup),
            "GLUP_s": round(lup / dt / 1e9, 2), "solves_per_s": round(count / dt, 2),
            "p50_problem_s": round(float(np.percentile(secs, 50)), 4),
            "p99_problem_s": round(float(np.percentile(secs, 99)), 4),
            "max_relres": max(i["relres"] for i in infos)}


def bench_adjoint(torch, srj, workloads, n=2048, levels=9, tol=1e-10):
    """Differentiable solve on 2048^2: forward SRJ and the adjoint SRJ backward."""
    from paper_1511_04292_amd.autograd import srj_solve_diff

    # untimed warm-up of the same forward and backward on a 64^2 copy of the workload: the
    # first backward of a process starts torch's autograd device thread and loads the kernels
    # of the loss and its gradient, tens of milliseconds that are no part of the solve
    ws = workloads.adjoint_2d(64)
    fs = torch.from_numpy(ws["f"]).to("cuda:0").requires_grad_(True)
    gs = torch.from_numpy(ws["g"]).to("cuda:0").requires_grad_(True)
    us = srj_solve_diff(fs, gs, srj.srj_plan((64, 64), ws["h"], P=3), tol=tol, tol_backward=1e-9)
    (0.5 * ((us - torch.from_numpy(ws["u_target"]).to("cuda:0"))[1:-1, 1:-1] ** 2).sum()).backward()
    torch.cuda.synchronize()
    del ws, fs, gs, us

    wl = workloads.adjoint_2d(n)
    f = torch.from_numpy(wl["f"]).to("cuda:0").requires_grad_(True)
    g = torch.from_numpy(wl["g"]).to("cuda:0").requires_grad_(True)
    ut = torch.from_numpy(wl["u_target"]).to("cuda:0")
    plan = srj.srj_plan((n, n), wl["h"], P=levels)
    tuned = srj.srj_plan_tune(plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = srj_solve_diff(f, g, plan, tol=tol, tol_backward=1e-9)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss = 0.5 * ((u - ut)[1:-1, 1:-1] ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fi, bi = u.grad_fn.info, u.grad_fn.backward_info
    pts = n * n

    fuse = int(tuned["fused_sweeps"])

    def rates(info):
        # effective per-sweep bytes: 24 B per point per sweep (above the HBM peak through the
        # fusion of sweeps); per launch (fused sweeps sharing one pass) a rate above the HBM
        # peak would mean the 101 MB working set is served from the 256 MB memory-side cache
        gbs = B_PER_POINT_F64 * pts * info["sweeps"] / info["seconds"] / 1e9
        per_launch = gbs / max(fuse, 1)
        return {"sweeps": int(info["sweeps"]), "device_s": round(info["seconds"], 4),
                "GLUP_s": round(pts * info["sweeps"] / info["seconds"] / 1e9, 1),
                "effective_per_sweep_GBs": round(gbs, 1), "per_launch_GBs": round(per_launch, 1),
                "per_launch_above_hbm_peak": per_launch > HBM_PEAK_GBS}

    return {"workload": f"2D {n}^2, f blobs and U(-1,1) ring as parameters, L = 1/2 ||u - u_target||^2, "
                        f"SRJ P={levels} forward to {tol:g}, adjoint to 1e-9 (binary64 floor of a smooth "
                        f"right-hand side is about 2e-10 here)",
            "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4), "launch_tuning": tuned,
            "forward": rates(fi), "backward": rates(bi), "loss": float(loss.detach())}


if __name__ == "__main__":
    main()
