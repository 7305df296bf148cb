"""Benchmark: whole optimal-control solves on one MI355X.

One step = one complete solve of the workload (right-hand side assembly, the
preconditioned Krylov solve to a 1e-8 true relative residual, recovery of y
and p), inputs resident in HBM.  Prints one JSON line.

Default workload: 2D heat tracking on the unit square, a = 1, M = 255
(h = 1/256), n = 256 steps, T = 1, theta = 1/2 (Crank-Nicolson),
gamma = 1e-4, seeded smooth modes + N(0, 1e-3) noise in f and g,
GMRES(30) with the block omega-circulant preconditioner P_S (zeta = pi), FP64.

Also measured in the same run:
  * per-kernel HIP-event timings over the timed region (library tracing);
    the roofline entry is the kernel family with the largest share of time,
    achieved = algorithmic bytes / duration, against the 8 TB/s HBM peak;
  * the preconditioner apply alone (five passes), model bytes / time;
  * cpu_baseline: the CPU oracle on a bounded sample of the same workload
    (two GMRES iterations on the full-size problem, scaled to the GPU's
    iteration count).

Usage: python bench.py [--steps K] [--warmup W] [--gamma G] [--precision fp64|mixed]
                       [--method gmres_ps|minres_abs_ps|minres_pms] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=int, default=2)
    ap.add_argument("--M", type=int, default=255)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--gamma", type=float, default=1e-4)
    ap.add_argument("--method", default="gmres_ps")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--pc-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(args, d, gpu_iters):
    """Oracle timed on this host: setup + rhs + `cpu_iters` Krylov iterations on the
    full-size problem, scaled linearly to the GPU's iteration count."""
    import numpy as np
    from oracle.discretization import Problem, AllAtOnce, rhs_tilde, transformed_rhs
    from oracle.precond import FastPreconditioner
    from oracle import krylov, solver as osolver
    kind, symmetric = osolver.METHODS[args.method]
    pr = Problem(dims=args.dims, M=args.M, n=args.n, theta=args.theta, gamma=args.gamma)
    t0 = time.perf_counter()
    op = AllAtOnce(pr)
    gt, ft = rhs_tilde(pr, d["f"], d["g"], d["y0"])
    b = transformed_rhs(pr, gt, ft, symmetric)
    P = FastPreconditioner(pr, kind)
    t1 = time.perf_counter()
    k = max(1, args.cpu_iters)
    if symmetric:
        krylov.minres(op.A, b, P.apply, tol=1e-30, maxit=k)
    else:
        krylov.gmres(op.Ahat, b, P.apply, tol=1e-30, restart=args.restart, maxit=k)
    t2 = time.perf_counter()
    x = np.zeros_like(b)
    osolver.recover(pr, x)
    t3 = time.perf_counter()
    per_iter = (t2 - t1) / k
    est_s = (t1 - t0) + (t3 - t2) + per_iter * max(gpu_iters, 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": round(est_s * 1000.0, 1), "unit": "ms per solve", "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle setup+rhs+recovery plus {k} Krylov iterations on the full-size "
                   f"workload ({per_iter:.2f} s/iteration), scaled to the GPU's {gpu_iters} "
                   f"iterations; host {os.cpu_count()} logical CPUs"),
        "measured_s": round(t3 - t0, 2),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the solver has no "
              "multi-GPU path in this build", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import datagen
    from paper_2406_00952_amd import wc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    d = datagen.config_problem(args.dims, args.M, args.n, seed=args.seed, noise_sigma=1e-3)
    m = args.M ** args.dims
    n = args.n
    f = torch.from_numpy(d["f"]).to(dev)
    g = torch.from_numpy(d["g"]).to(dev)
    y0 = torch.from_numpy(d["y0"]).to(dev)
    y = torch.empty(n * m, dtype=torch.float64, device=dev)
    p = torch.empty_like(y)
    plan = wc.Plan(args.dims, args.M, n, theta=args.theta, gamma=args.gamma, method=args.method,
                   precision=args.precision, restart=args.restart, tol=1e-8, maxit=500)
    log(f"plan footprint {plan.footprint / 2**30:.2f} GiB")
    for i in range(args.warmup):
        info = plan.solve(f, g, y0, y, p)
        log(f"warmup {i}: iters {info.iters} relres {info.relres:.2e} {info.ms:.1f} ms")
    # ---- timed region (kernel tracing on) -----------------------------------
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(plan.solve(f, g, y0, y, p))
        log(f"step {i}: iters {infos[-1].iters} relres {infos[-1].relres:.2e} {infos[-1].ms:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.profile(False)
    stats = plan.profile_read()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    iters = infos[-1].iters
    relres = max(i.relres for i in infos)

    # ---- preconditioner apply alone ------------------------------------------
    v = torch.randn(2 * n * m, dtype=torch.float64, device=dev)
    w = torch.empty_like(v)
    for _ in range(3):
        plan.pc_apply(v, w)
    plan.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.pc_reps):
        plan.pc_apply(v, w)
    e1.record()
    torch.cuda.synchronize()
    plan.profile(False)
    pc_stats = plan.profile_read()
    pc_ms = e0.elapsed_time(e1) / args.pc_reps
    es = 16 if args.precision == "fp64" else 8
    nvec = 2 * n * m
    if args.dims == 2:
        pc_bytes = nvec * (8 + es // 2) * 2 + 3 * 2 * nvec * (es // 2)
    else:
        pc_bytes = nvec * (8 + es // 2) * 2 + 2 * nvec * (es // 2)
    pc_gbs = pc_bytes / (pc_ms * 1e-3) / 1e9

    # ---- roofline: dominant kernel family of the timed region -----------------
    fam = {k: v for k, v in stats.items() if v[0] > 0}
    dom = max(fam, key=lambda k: fam[k][1])
    launches, tot_ms, tot_bytes = fam[dom]
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] * 1000.0 / v[0], 2),
                   "share": round(v[1] / sum(x[1] for x in fam.values()), 4),
                   "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in sorted(fam.items(), key=lambda kv: -kv[1][1])}
    pc_kernels = {k: {"avg_us": round(v[1] * 1000.0 / v[0], 2),
                      "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1)}
                  for k, v in pc_stats.items() if v[0] > 0}

    out = {
        "metric": "solve ms to 1e-8 rel. residual; PC-apply HBM GB/s; p50/p99 served latency",
        "value": round(ms_per_step, 3),
        "unit": "ms per solve",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 Krylov / f32 preconditioner",
        "data": "synthetic",
        "config": {"workload": f"heat{args.dims}d_M{args.M}_n{args.n}",
                   "dims": args.dims, "M": args.M, "n": n, "theta": args.theta,
                   "gamma": args.gamma, "zeta": "pi", "method": args.method,
                   "precision": args.precision, "restart": args.restart, "tol": 1e-8,
                   "dof": 2 * n * m, "seed": args.seed},
        "iters": iters, "relres": relres, "reorth": infos[-1].reorth,
        "solves_per_s": round(1000.0 / ms_per_step, 3),
        "pc_apply": {"ms": round(pc_ms, 4), "model_bytes": pc_bytes, "GBps": round(pc_gbs, 1),
                     "frac_of_peak": round(pc_gbs / HBM_PEAK_GBS, 4), "kernels": pc_kernels},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "avg_us": round(tot_ms * 1000.0 / launches, 2),
                     "bytes_per_launch": tot_bytes / launches},
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args, d, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
