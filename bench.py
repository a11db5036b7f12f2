#!/usr/bin/env python
"""Benchmark of the SA-AMG preconditioned CG Poisson solve on one MI355X.

A step is one complete solve to relative residual 1e-8 (scaled system) from x0 = 0,
reusing the preconditioner built once before the warm-up (the paper's "reusing the
preconditioner" mode), on the 256 x 256 x 768 elliptic pipe (semi-axes 1.0 x 0.6,
length 4, 39.1M unknowns, quadratic wall rule) with a seeded 1M-particle Gaussian
bunch deposited by cloud-in-cell.  The headline value is DOF*iter/s of the mixed
path (fp32 hierarchy / fp64 CG); the all-fp64 path is run on the same right-hand side
and reported beside it, and a short served stream of mixed pipe requests (Poisson
arrivals) gives p50/p99 latency for both precisions.  Setup time is reported
separately (the paper's "construction").

The roofline figure is for the kernel class with the largest share of solve time: a
breakdown pass times every class, then the timed solves run with HIP events on that
class only.  Its HBM traffic comes from the committed rocprofv3 counter summary when
that summary was taken on the current kernel sources.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ell256_mixed",
                    help="workloads.by_name key (default: the 256x256x768 ellipse, mixed)")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timers", action="store_true",
                    help="time without per-kernel HIP events (roofline omitted)")
    ap.add_argument("--cpu-sample-planes", type=int, default=160)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="served-stream mode: Poisson arrivals of mixed pipe requests")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--pic", action="store_true",
                    help="PIC sequence: moving bunch, one hierarchy, warm-started solves")
    ap.add_argument("--pic-steps", type=int, default=20)
    ap.add_argument("--no-variants", action="store_true",
                    help="headline mode: skip the Gauss-Seidel coarse-solver leg")
    ap.add_argument("--no-serve", action="store_true",
                    help="headline mode: skip the short served-stream leg (p50/p99 latency)")
    ap.add_argument("--line-serve-requests", type=int, default=32,
                    help="requests in the headline mode's served-stream leg")
    ap.add_argument("--paper-tubes", action="store_true",
                    help="the paper's tube problems (Tables 8-10) with open ends, one GPU")
    ap.add_argument("--tube-sizes", default="256,512,1024")
    ap.add_argument("--tube-reps", type=int, default=2)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="open-loop arrival rate as a fraction of the closed-loop solves/s")
    ap.add_argument("--serve-setup-workers", type=int, default=None,
                    help="threads building hierarchies of new geometries (server default if unset)")
    return ap.parse_args()


def pic_bench(args) -> dict:
    """Successive PIC steps on the 192x192x1024 cylinder (L = 8) as a 2M-particle bunch moves
    0.02 along z per step.  Each step deposits the bunch on the GPU (cloud-in-cell), solves
    with the hierarchy built once, starting from the previous solution (Section 4: previous
    time step as initial guess; Section 5: reuse of the preconditioner), and gathers
    E = -grad(phi) back to the particles.  The rigid shift of the bunch stands in for the
    particle push and is not timed."""
    import torch

    import paper_0907_4863_amd as sa
    import workloads as W

    w = W.c5_cylinder192(sa.MIXED)
    dev = torch.device("cuda:0")
    dom = sa.domain_for(w.shape, w.nx, w.ny, w.nz)
    base = torch.from_numpy(W.draw_particles(w.bunch)).to(dev)
    n = base.shape[0]
    origin = (-w.shape.a, -w.shape.b, -0.5 * w.shape.length)
    t0 = time.perf_counter()
    H = sa.setup(dom, w.variant, sa.default_options(precision=sa.MIXED))
    P = sa.pic_create(dom, origin, n)
    torch.cuda.synchronize()
    setup_ms = 1e3 * (time.perf_counter() - t0)
    xa = torch.zeros(w.box_nodes, dtype=torch.float64, device=dev)
    xb = torch.zeros_like(xa)
    rho = torch.zeros_like(xa)
    E = torch.empty_like(base)
    steps = []
    for k in range(args.pic_steps):
        pos = base.clone()
        pos[:, 2] += W.pic_shift(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sa.pic_deposit(P, pos, 1.0 / n, rho)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = sa.solve(H, rho, xb, x0=(xa if k > 0 else None), tol=w.tol)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sa.pic_gather(P, xb, pos, E)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        steps.append((res["iterations"], 1e3 * (t2 - t1), res["rel_res_true"], 1e3 * (t1 - t0),
                      1e3 * (t3 - t2)))
        xa, xb = xb, xa
        print(f"[bench] pic step {k}: deposit {1e3 * (t1 - t0):.2f} ms, solve {res['iterations']} it "
              f"{1e3 * (t2 - t1):.1f} ms, gather {1e3 * (t3 - t2):.2f} ms", file=sys.stderr, flush=True)
    sa.pic_destroy(P)
    sa.destroy(H)
    later = steps[1:] if len(steps) > 1 else steps
    it_l = sum(s[0] for s in later)
    ms_l = sum(s[1] for s in later)
    return {"workload": "cylinder R=1 L=8 192x192x1024, linear wall rule, mixed, 2M particles",
            "dof": dom.n_unknowns, "particles": n, "setup_ms": setup_ms, "steps": len(steps),
            "first_step": {"iterations": steps[0][0], "ms": steps[0][1]},
            "warm_steps_mean_iterations": it_l / len(later),
            "warm_steps_mean_ms": ms_l / len(later),
            "warm_dof_iter_per_s": dom.n_unknowns * it_l / (ms_l * 1e-3),
            "deposit_ms_mean": sum(s[3] for s in steps) / len(steps),
            "gather_ms_mean": sum(s[4] for s in steps) / len(steps),
            "pic_step_ms_mean": sum(s[1] + s[3] + s[4] for s in later) / len(later),
            "max_rel_res": max(s[2] for s in steps)}


# The paper's tube problems (Section 5.3, Tables 8-10): a circular tube inscribed in an n^3
# lattice with open (Robin) ends, all n planes unknown.  "paper" holds the fastest
# solution and construction times printed for each, on the Cray XT4/XT3 (Opteron 2.6 GHz).
PAPER_TUBES = [
    {"n": 256, "variant": "lin", "table": "Table 8",
     "paper": {"cores": 512, "solution_s": 0.71, "construction_s": 0.83}},
    {"n": 512, "variant": "const", "table": "Table 9",
     "paper": {"cores": 2048, "solution_s": 2.54, "construction_s": 7.58}},
    {"n": 1024, "variant": "lin", "table": "Table 10",
     "paper": {"cores": 2048, "solution_s": 10.93, "construction_s": 6.68}},
]


def tube_bench(args) -> dict:
    """Setup and solve of each tube on one GPU, mixed and fp64 (x0 = 0, rel-res 1e-8)."""
    import torch

    import paper_0907_4863_amd as sa
    import workloads as W

    dev = torch.device("cuda:0")
    sizes = [int(v) for v in args.tube_sizes.split(",")]
    out = []
    for spec in PAPER_TUBES:
        n = spec["n"]
        if n not in sizes:
            continue
        variant = {"const": W.VARIANT_CONST, "lin": W.VARIANT_LIN}[spec["variant"]]
        shape = W.Shape.cylinder(1.0, 2.0)
        w = W.Workload(f"tube{n}", shape, n, n, n, variant, W.PREC_MIXED,
                       bunch=W.Bunch(1_000_000, (0.1, 0.1, 0.3), seed=7), robin=True)
        t0 = time.perf_counter()
        dom = sa.domain_for(shape, n, n, n, open_ends=True)
        t_dom = time.perf_counter() - t0
        print(f"[bench] tube {n}^3: domain built in {t_dom:.1f} s, depositing the bunch",
              file=sys.stderr, flush=True)
        b_host = W.rhs(w)
        b = torch.from_numpy(b_host.reshape(-1)).to(dev)
        del b_host
        print(f"[bench] tube {n}^3: {dom.n_unknowns} unknowns, host domain {t_dom:.1f} s",
              file=sys.stderr, flush=True)
        rec = {"table": spec["table"], "grid": f"{n}^3", "wall_rule": spec["variant"],
               "unknowns": dom.n_unknowns, "host_domain_s": t_dom, "paper": spec["paper"]}
        for tag, prec in (("mixed", sa.MIXED), ("fp64", sa.FP64)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = sa.setup(dom, variant, sa.default_options(precision=prec))
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            x = torch.zeros(w.box_nodes, dtype=torch.float64, device=dev)
            res = sa.solve(H, b, x, tol=1e-8, max_iter=500)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = args.tube_reps
            for _ in range(reps):
                res = sa.solve(H, b, x, tol=1e-8, max_iter=500)
            torch.cuda.synchronize()
            t_solve = (time.perf_counter() - t0) / reps
            info = sa.hierarchy_info(H)
            rec[tag] = {"setup_s": t_setup, "solve_s": t_solve, "iterations": res["iterations"],
                        "status": res["status"], "rel_res_true": res["rel_res_true"],
                        "dof_iter_per_s": dom.n_unknowns * res["iterations"] / t_solve,
                        "levels": info["n_unknowns"], "device_bytes": info["device_bytes"]}
            print(f"[bench] tube {n}^3 {tag}: setup {t_setup:.2f} s, solve {t_solve:.3f} s, "
                  f"{res['iterations']} it, status {res['status']}", file=sys.stderr, flush=True)
            sa.destroy(H)
            del x
            torch.cuda.empty_cache()
        del b
        torch.cuda.empty_cache()
        out.append(rec)
    return {"tubes": out}


def serve_bench(args, n_requests=None) -> dict:
    """Continuous batching over a seeded stream of pipe solves (cylinder, ellipse and
    box-with-bore; cross-section edge 32..160; length ratio 1..4).  After an untimed warm-up
    on the first 8 requests in each precision, pass 1 admits every request at t = 0 (closed
    loop) to measure capacity, in mixed precision and in fp64; then Poisson arrivals at
    serve_load x the mixed capacity are replayed in mixed precision and in fp64."""
    import dataclasses as dc

    import paper_0907_4863_amd as sa
    import workloads as W
    from paper_0907_4863_amd import serve

    reqs = W.serving_stream(n_requests=n_requests or args.serve_requests, qps=1.0, seed=4)
    print(f"[bench] serve: generating {len(reqs)} right-hand sides", file=sys.stderr, flush=True)
    rhs = {}
    for k, r in enumerate(reqs):
        rhs[r.rid] = W.rhs(r.workload)
        if (k + 1) % 64 == 0:
            print(f"[bench] serve: {k + 1} right-hand sides", file=sys.stderr, flush=True)
    dof_total = 0
    out = {}

    def run(tag, arrivals, precision, subset=None):
        rs = [W.Request(r.rid, t, dc.replace(r.workload, precision=precision))
              for r, t in zip(subset or reqs, arrivals)]
        cfg = serve.ServeConfig(precision=precision, max_active=16, hbm_budget_bytes=200 << 30)
        if getattr(args, "serve_setup_workers", None):
            cfg.setup_workers = args.serve_setup_workers
        srv = serve.Server(cfg, serve.GpuEngine())
        recs = srv.run(rs, rhs_of=lambda q: rhs[q.rid])
        srv.close()
        summ = serve.summarize(recs)
        summ["max_concurrent"] = srv.max_concurrent
        summ["peak_device_bytes"] = srv.peak_used
        print(f"[bench] serve {tag}: {summ}", file=sys.stderr, flush=True)
        return summ

    # untimed: the first requests once in each precision, so that no timed pass pays the
    # first use of the allocator's pool, the streams and the kernels
    nw = min(8, len(reqs))
    for prec in (sa.MIXED, sa.FP64):
        run("warm-up", [0.0] * nw, prec, subset=reqs[:nw])
    closed = run("closed-loop mixed", [0.0] * len(reqs), sa.MIXED)
    out["closed_loop_fp64"] = run("closed-loop fp64", [0.0] * len(reqs), sa.FP64)
    qps = args.serve_load * closed["solves_per_s"]
    gaps = np.random.default_rng(4).exponential(1.0 / qps, size=len(reqs))
    arr = list(np.cumsum(gaps) - gaps[0])
    out["closed_loop_mixed"] = closed
    out["open_loop_mixed"] = run("open-loop mixed", arr, sa.MIXED)
    out["open_loop_fp64"] = run("open-loop fp64", arr, sa.FP64)
    out["qps"] = qps
    return out


def hbm_ceiling() -> dict:
    """Best rates of the device's own streaming kernels (paper_0907_4863_amd/hbm_ceiling,
    built by build(): 16-byte copy / read / write over 2 GiB, ordinary and nontemporal),
    in GB/s, and the runtime's device-to-device copy.  Run as a child process."""
    exe = os.path.join(ROOT, "paper_0907_4863_amd", "hbm_ceiling")
    if not os.path.exists(exe):
        return {}
    res = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    best = {}
    for ln in res.stdout.splitlines():
        parts = ln.split()
        if ln.startswith("blocks") and len(parts) >= 7:
            best[parts[2]] = max(best.get(parts[2], 0.0), float(parts[5]))
        elif ln.startswith("hipMemcpy"):
            best["hipMemcpy_d2d"] = float(parts[4])
    return {f"{k}_GBs": v for k, v in best.items()}


def _kernel_sources_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("fine.hip", "wide.hip", "coarse.hip", "common.h", "launch.h", "march.h"):
        with open(os.path.join(ROOT, "paper_0907_4863_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None when no summary
    exists or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for ln in fh:
            parts = ln.split()
            if len(parts) == 2 and not ln.startswith("#"):
                rec[parts[0]] = parts[1]
    if rec.get("sources_sha256") != _kernel_sources_digest():
        return None
    try:
        return float(rec["fetch_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def oracle_check(w, solutions: dict) -> dict:
    """Each GPU solution against the oracle: the scaled true residual D^-1/2 (b - A x) that
    the oracle's own operator gives on every row (matrix-free, fp64), relative to ||b~||;
    the stopping rule asks for <= tol.  The oracle cannot solve this size in a bench."""
    import workloads as W
    from oracle import grid, operator

    t0 = time.perf_counter()
    dom = grid.from_shape(w.shape, w.nx, w.ny, w.nz)
    b = W.rhs(w)
    out = {}
    for tag, x in solutions.items():
        r, bn = operator.scaled_residual(dom, w.variant, x, b)
        out[tag] = float(np.linalg.norm(r) / bn)
    out["rows"] = int(dom.n_unknowns)
    out["check_s"] = time.perf_counter() - t0
    return out


def cpu_baseline(w, planes: int) -> dict:
    """The oracle, single-threaded, on a z-slab of the same pipe cross-section and spacing."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import solve

    L = w.shape.length * (planes - 1) / (w.nz - 1)
    shape = W.Shape(w.shape.kind, w.shape.a, w.shape.b, L, w.shape.bore_r, w.shape.cavity_half_len)
    bunch = W.Bunch(w.bunch.n, (w.bunch.sigma[0], w.bunch.sigma[1], L / 6.0), w.bunch.seed)
    ws = W.Workload("sample", shape, w.nx, w.ny, planes, w.variant, W.PREC_FP64, bunch=bunch)
    b = W.rhs(ws)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sys_, H = solve.build(shape, w.nx, w.ny, planes, w.variant)
        t1 = time.perf_counter()
        res = solve.solve(sys_, H, b, tol=w.tol)
        t2 = time.perf_counter()
    dof = sys_.n
    return {
        "value": dof * res.iterations / (t2 - t1),
        "unit": "DOF*iter/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"oracle (numpy/scipy fp64, 1 thread) on a {w.nx}x{w.ny}x{planes} slab of the "
                   f"same pipe (same spacing, {dof} unknowns): setup {t1 - t0:.2f} s, "
                   f"{res.iterations} iterations in {t2 - t1:.2f} s"),
        "setup_s": t1 - t0,
        "solve_s": t2 - t1,
        "iterations": res.iterations,
        "host_cpu": _cpu_model(),
        "host_threads": os.cpu_count(),
    }


def run_solves(sa, torch, H, b, nbox, steps, warmup, dev, timers: bool):
    """Warm-up, then (timers) a per-kernel-class breakdown pass, then the timed solves.

    The timed region runs with HIP-event timing on the dominant kernel class only, so its
    average launch duration is measured live while the other launches carry no events."""
    x = torch.zeros(nbox, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        sa.solve(H, b, x, tol=1e-8, max_iter=500)
    torch.cuda.synchronize()

    def read_timers(kinds):
        out = {}
        for k in kinds:
            ms, n, byts = sa.capi.timer_read(k)
            if n:
                out[k] = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / n,
                          "alg_bytes_per_launch": byts / n,
                          "achieved_GBs": byts / (ms * 1e-3) / 1e9 if ms > 0 else None}
        return out

    kern, dom_k = {}, None
    if timers:
        sa.capi.timer_reset()
        for k in sa.capi.TIMER_KINDS:
            sa.capi.timer_enable(k, True)
        for _ in range(2):
            sa.solve(H, b, x, tol=1e-8, max_iter=500)
        torch.cuda.synchronize()
        for k in sa.capi.TIMER_KINDS:
            sa.capi.timer_enable(k, False)
        kern = read_timers(sa.capi.TIMER_KINDS)
        sa.capi.timer_reset()
        dom_k = max(kern, key=lambda k: kern[k]["total_ms"])
        sa.capi.timer_enable(dom_k, True)
    iters = []
    res = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = sa.solve(H, b, x, tol=1e-8, max_iter=500)
        iters.append(res["iterations"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    live = None
    if timers:
        sa.capi.timer_enable(dom_k, False)
        live = read_timers([dom_k]).get(dom_k)
        if live is not None:
            live["kernel"] = dom_k
        sa.capi.timer_reset()
    return x, iters, wall, res, kern, live


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this solver runs on a single GPU "
              f"(one solve per device). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_0907_4863_amd as sa
    import workloads as W

    if args.pic:
        res = pic_bench(args)
        print(json.dumps({
            "metric": "DOF*iter/s of warm-started PIC solves at rel-res 1e-8",
            "value": res["warm_dof_iter_per_s"], "unit": "DOF*iter/s", "n_gpus": 1,
            "steps": res["steps"], "warmup": 0, "ms_per_step": res["warm_steps_mean_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic (seeded 2M-particle bunch, cloud-in-cell)",
            "config": {"workload": res["workload"], "dof": res["dof"]}, "pic": res}), flush=True)
        return
    if args.paper_tubes:
        res = tube_bench(args)
        big = res["tubes"][-1]
        print(json.dumps({
            "metric": "solution time of the paper's open-ended tube problems on one GPU "
                      "(rel-res 1e-8, x0 = 0, preconditioner built once)",
            "value": big["mixed"]["solve_s"], "unit": "s", "n_gpus": 1,
            "steps": args.tube_reps, "warmup": 1, "ms_per_step": 1e3 * big["mixed"]["solve_s"],
            "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic (seeded 1M-particle Gaussian bunch, cloud-in-cell)",
            "config": {"workload": f"tube {big['grid']}, {big['wall_rule']} wall rule, open ends, "
                                   f"{big['unknowns']} unknowns"},
            **res}), flush=True)
        return
    if args.serve:
        res = serve_bench(args)
        m, f = res["open_loop_mixed"], res["open_loop_fp64"]
        print(json.dumps({
            "metric": "served solves/s and p50/p99 latency at rel-res 1e-8 (Poisson arrivals)",
            "value": m["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.serve_requests, "warmup": 0, "ms_per_step": 1e3 / m["solves_per_s"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64", "data": "synthetic (seeded Gaussian bunches, cloud-in-cell)",
            "config": {"workload": f"served stream of {args.serve_requests} pipe solves "
                                   f"(cylinder/ellipse/box-with-bore, edge 32..160, ratio 1..4), "
                                   f"Poisson arrivals at {res['qps']:.2f}/s"},
            "p50_latency_ms": m["p50_latency_ms"], "p99_latency_ms": m["p99_latency_ms"],
            "warm_up": "first 8 requests once in each precision, untimed",
            "fp64": f, "closed_loop_mixed": res["closed_loop_mixed"],
            "closed_loop_fp64": res["closed_loop_fp64"], "open_loop_mixed": m,
        }), flush=True)
        return

    w = W.by_name(args.workload)
    ceiling = hbm_ceiling()
    print(f"[bench] HBM streaming ceilings (GB/s): {ceiling}", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    if args.copy_mb:
        n = args.copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.copy_mb} MiB done", file=sys.stderr, flush=True)
        del src, dst
    print(f"[bench] workload {w.name} {w.nx}x{w.ny}x{w.nz}", file=sys.stderr, flush=True)
    dom = sa.domain_for(w.shape, w.nx, w.ny, w.nz)
    dof = dom.n_unknowns
    b = torch.from_numpy(W.rhs(w).reshape(-1)).to(dev)
    nbox = w.box_nodes
    out = {}
    for tag, prec in (("mixed", sa.MIXED), ("fp64", sa.FP64)):
        if w.precision == sa.FP64 and tag == "mixed":
            continue
        if args.skip_fp64 and tag == "fp64" and w.precision == sa.MIXED:
            continue
        steps = args.steps if tag == ("mixed" if w.precision == sa.MIXED else "fp64") else \
            (args.fp64_steps if args.fp64_steps is not None else max(1, args.steps // 2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = sa.setup(dom, w.variant, sa.default_options(precision=prec))
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        info = sa.hierarchy_info(H)
        print(f"[bench] {tag}: setup {setup_s:.3f} s levels {info['n_unknowns']}",
              file=sys.stderr, flush=True)
        # the same setup again, once the process's pool and kernels are warm (a server
        # building its next hierarchy)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H2 = sa.setup(dom, w.variant, sa.default_options(precision=prec))
        torch.cuda.synchronize()
        setup_warm_s = time.perf_counter() - t0
        sa.destroy(H2)
        x, iters, wall, res, kern, live = run_solves(sa, torch, H, b, nbox, steps, args.warmup,
                                                     dev, timers=not args.no_timers)
        out[tag] = {"x": x, "iters": iters, "wall": wall, "res": res, "kern": kern, "live": live,
                    "setup_s": setup_s, "setup_warm_s": setup_warm_s, "info": info,
                    "steps": steps}
        print(f"[bench] {tag}: {steps} solves in {wall:.3f} s, iterations {iters}",
              file=sys.stderr, flush=True)
        sa.destroy(H)

    head = out["mixed"] if "mixed" in out else out["fp64"]
    total_iters = sum(head["iters"])
    value = dof * total_iters / head["wall"]
    line = {
        "metric": "DOF\u00b7iter/s and solves/s at rel-res 1e-8 (FP32-AMG vs FP64); p50/p99 latency",
        "value": value,
        "unit": "DOF*iter/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["wall"] / head["steps"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if "mixed" in out else "f64",
        "data": "synthetic (seeded Gaussian bunch, cloud-in-cell)",
        "config": {"workload": f"{w.name}: ellipse 1.0x0.6 L={w.shape.length} "
                               f"{w.nx}x{w.ny}x{w.nz} box, {dof} unknowns, "
                               f"{W.VARIANT_NAMES[w.variant]} wall rule, rel-res {w.tol}",
                   "dof": dof, "levels": head["info"]["n_unknowns"]},
        "solves_per_s": head["steps"] / head["wall"],
        "iterations": head["iters"][-1],
        "setup_ms": 1e3 * head["setup_s"],
        "setup_warm_ms": 1e3 * head["setup_warm_s"],
        "rel_res_true": head["res"]["rel_res_true"],
    }
    if "fp64" in out and "mixed" in out:
        f = out["fp64"]
        xm = out["mixed"]["x"]
        xf = f["x"]
        line["fp64"] = {
            "value": dof * sum(f["iters"]) / f["wall"],
            "ms_per_step": 1e3 * f["wall"] / f["steps"],
            "solves_per_s": f["steps"] / f["wall"],
            "iterations": f["iters"][-1],
            "setup_ms": 1e3 * f["setup_s"],
            "setup_warm_ms": 1e3 * f["setup_warm_s"],
            "rel_res_true": f["res"]["rel_res_true"],
        }
        line["mixed_vs_fp64_rel_err"] = float(torch.linalg.norm(xm - xf) / torch.linalg.norm(xf))
    kern, live = head["kern"], head["live"]
    if live:
        dom_k = live["kernel"]
        line["roofline"] = {
            "kernel": dom_k,
            "bound": "hbm",
            "achieved": live["achieved_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": live["achieved_GBs"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom_k, w.name),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_us": live["avg_us"],
            "launches": live["launches"],
            "alg_bytes_per_launch": live["alg_bytes_per_launch"],
            "measured_ceilings_GBs": ceiling,
        }
        line["kernels"] = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                               for kk, vv in v.items()} for k, v in kern.items()}
    if not args.no_variants and "mixed" in out:
        # the paper's iterative coarse level solver (3 Gauss-Seidel sweeps) on the same b
        t0 = time.perf_counter()
        H = sa.setup(dom, w.variant, sa.default_options(precision=sa.MIXED,
                                                         coarse_solver=sa.COARSE_GS))
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        x = torch.zeros(nbox, dtype=torch.float64, device=dev)
        sa.solve(H, b, x, tol=1e-8, max_iter=500)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            rg = sa.solve(H, b, x, tol=1e-8, max_iter=500)
        torch.cuda.synchronize()
        t_solve = (time.perf_counter() - t0) / reps
        sa.destroy(H)
        line["coarse_gauss_seidel"] = {
            "coarse_solver": "3 Gauss-Seidel sweeps (mixed path; direct solve is the default)",
            "setup_ms": 1e3 * t_setup, "ms_per_step": 1e3 * t_solve,
            "iterations": rg["iterations"], "rel_res_true": rg["rel_res_true"],
            "value": dof * rg["iterations"] / t_solve}
        print(f"[bench] coarse Gauss-Seidel: setup {1e3 * t_setup:.1f} ms, "
              f"{1e3 * t_solve:.2f} ms per solve, {rg['iterations']} it", file=sys.stderr, flush=True)
        del x
        # reuse of the aggregation hierarchy (Section 5.2): the bunch elongates, so h_z
        # grows while the lattice and its unknowns stay; numeric-only re-setups of one
        # hierarchy against fresh setups of the same domains
        import dataclasses
        H = sa.setup(dom, w.variant, sa.default_options(precision=sa.MIXED))
        Hp = sa.setup(dom, w.variant, sa.default_options(precision=sa.MIXED))
        t_refresh, t_fresh, it_refresh, it_fresh = [], [], [], []
        t_op, it_op = [], []
        x = torch.zeros(nbox, dtype=torch.float64, device=dev)
        for grow in (1.05, 1.10, 1.15):
            d2 = sa.domain_for(dataclasses.replace(w.shape, length=w.shape.length * grow),
                               w.nx, w.ny, w.nz)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sa.refresh(H, d2)
            torch.cuda.synchronize()
            t_refresh.append(time.perf_counter() - t0)
            it_refresh.append(sa.solve(H, b, x, tol=w.tol, max_iter=500)["iterations"])
            # reuse of the preconditioner: the original one, the new operator
            t0 = time.perf_counter()
            sa.set_operator(Hp, d2)
            torch.cuda.synchronize()
            t_op.append(time.perf_counter() - t0)
            it_op.append(sa.solve(Hp, b, x, tol=w.tol, max_iter=500)["iterations"])
            t0 = time.perf_counter()
            F = sa.setup(d2, w.variant, sa.default_options(precision=sa.MIXED))
            torch.cuda.synchronize()
            t_fresh.append(time.perf_counter() - t0)
            it_fresh.append(sa.solve(F, b, x, tol=w.tol, max_iter=500)["iterations"])
            sa.destroy(F)
        torch.cuda.synchronize()
        sa.destroy(H)
        sa.destroy(Hp)
        del x
        line["hierarchy_reuse"] = {
            "workload": f"{w.name} with the length grown by 5, 10 and 15 % (h_z changes, "
                        f"same unknowns), mixed precision",
            "refresh_ms": [round(1e3 * t, 1) for t in t_refresh],
            "fresh_setup_ms": [round(1e3 * t, 1) for t in t_fresh],
            "refresh_over_setup": sum(t_refresh) / sum(t_fresh),
            "iterations_refreshed": it_refresh, "iterations_fresh": it_fresh,
            "preconditioner_reuse": {
                "what": "the original length's preconditioner kept, the operator of each "
                        "longer pipe set (saamg_set_operator)",
                "operator_update_ms": [round(1e3 * t, 1) for t in t_op],
                "iterations": it_op}}
        print(f"[bench] hierarchy reuse: refresh {[round(1e3 * t) for t in t_refresh]} ms vs "
              f"fresh setup {[round(1e3 * t) for t in t_fresh]} ms", file=sys.stderr, flush=True)
    if not args.no_serve:
        sv = serve_bench(args, n_requests=args.line_serve_requests)
        m, f = sv["open_loop_mixed"], sv["open_loop_fp64"]
        keep = ("requests", "completed", "solves_per_s", "p50_latency_ms", "p99_latency_ms",
                "mean_iterations", "max_concurrent", "cache_hits", "warm_starts",
                "mean_iterations_warm", "mean_iterations_cold")
        line["p50_latency_ms"] = m["p50_latency_ms"]
        line["p99_latency_ms"] = m["p99_latency_ms"]
        line["serving"] = {
            "workload": f"served stream of {m['requests']} pipe solves (cylinder/ellipse/"
                        f"box-with-bore, edge 32..160, ratio 1..4, linear rule), Poisson "
                        f"arrivals at {sv['qps']:.2f}/s = {args.serve_load} x closed-loop capacity",
            "warm_up": "first 8 requests once in each precision, untimed",
            "closed_loop_mixed_solves_per_s": sv["closed_loop_mixed"]["solves_per_s"],
            "closed_loop_fp64_solves_per_s": sv["closed_loop_fp64"]["solves_per_s"],
            "mixed": {k: m[k] for k in keep}, "fp64": {k: f[k] for k in keep}}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_planes)
        print("[bench] oracle residual of the GPU solutions ...", file=sys.stderr, flush=True)
        sols = {tag: out[tag]["x"].cpu().numpy() for tag in out}
        chk = oracle_check(w, sols)
        line["oracle_rel_res_true"] = {
            **{tag: chk[tag] for tag in sols},
            "definition": "||D^-1/2 (b - A x)|| / ||D^-1/2 b|| of each GPU solution with the "
                          "oracle's operator, over all rows (the stopping rule's quantity)",
            "rows": chk["rows"], "check_s": round(chk["check_s"], 1)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
