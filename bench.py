"""Benchmark: whole optimal-control solves on one MI355X.

One step = one complete solve of the workload (right-hand side assembly, the
preconditioned Krylov solve to a 1e-8 true relative residual, recovery of y
and p), inputs resident in HBM.  Prints one JSON line.

Default workload: 2D heat tracking on the unit square, a = 1, M = 255
(h = 1/256), n = 256 steps, T = 1, theta = 1/2 (Crank-Nicolson),
gamma = 1e-4, seeded smooth modes + N(0, 1e-3) noise in f and g,
GMRES(30) with the block omega-circulant preconditioner P_S (zeta = pi), FP64,
in the low-rank form (the Arnoldi process in the compact coordinates that the GMRES
proposition gives: same iterates, no full-length basis; --lowrank 0 for the
standard form).  Only GMRES-P_S in FP64 with a = 1 has that form; other methods,
precisions and coefficients run the standard form.

Also measured in the same run:
  * the standard form of the same solve (full-length basis, matvec each step);
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
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick the preconditioner tile widths by timing them first")
    ap.add_argument("--graphs", type=int, default=1,
                    help="replay captured Krylov iterations (not while tracing kernels)")
    ap.add_argument("--lowrank", type=int, default=1,
                    help="GMRES-P_S Arnoldi in the compact coordinates of the GMRES proposition")
    ap.add_argument("--standard-steps", type=int, default=3,
                    help="also time the standard GMRES form (full basis, matvec per step)")
    ap.add_argument("--flexible", type=int, default=1,
                    help="GMRES stores P^-1 v_j (same iterates; no final preconditioner apply)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mg-tol", type=float, default=1e-10,
                    help="multigrid cycle tolerance (variable a); 0 = exactly --mg-cycles cycles")
    ap.add_argument("--mg-cycles", type=int, default=30, help="multigrid cycle cap (variable a)")
    ap.add_argument("--coeff", choices=["const", "sin"], default="const",
                    help="a = 1, or a = 1 + 0.5 sin(2 pi x1) sin(2 pi x2) (multigrid)")
    ap.add_argument("--pc-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=5)
    ap.add_argument("--serve", action="store_true",
                    help="serving mode: Poisson arrivals of a mixed request population")
    ap.add_argument("--rates", default="5,20,60,150", help="arrival rates (requests/s), --serve")
    ap.add_argument("--requests", type=int, default=60, help="requests per rate, --serve")
    ap.add_argument("--concurrency", type=int, default=4, help="server workers, --serve")
    ap.add_argument("--batch", type=int, default=8,
                    help="instances of the small serving shape (2D, M=63, n=64) solved one by "
                         "one and as one batch (0 = skip)")
    return ap.parse_args()


def batch_bench(args):
    """Many instances of a small problem: sequential wc_solve (captured iterations) against
    one lockstep batch (one launch per preconditioner pass for all instances)."""
    import numpy as np
    import torch
    import datagen
    from paper_2406_00952_amd import wc
    M, n, k = 63, 64, args.batch
    plans = [wc.Plan(2, M, n, theta=0.5, gamma=1e-4, method="gmres_ps", tol=1e-8, maxit=500)
             for _ in range(k)]
    data = []
    for i in range(k):
        d = datagen.config_problem(2, M, n, seed=args.seed + 10 + i, noise_sigma=1e-3)
        data.append([torch.from_numpy(np.ascontiguousarray(d[x])).cuda() for x in ("f", "g", "y0")])
    ys = [torch.empty(n * M * M, dtype=torch.float64, device="cuda") for _ in range(k)]
    ps = [torch.empty_like(y) for y in ys]
    reps = 5

    def seq():
        return [pl.solve(*dd, y, p) for pl, dd, y, p in zip(plans, data, ys, ps)]

    batch = wc.Batch(plans)
    cols = [[dd[j] for dd in data] for j in range(3)]

    def bat():
        return batch.solve(cols[0], cols[1], cols[2], ys, ps)

    out = {"instances": k, "shape": "2D M=63 n=64 fp64 GMRES(30)-P_S"}
    for name, fn in (("sequential", seq), ("batch", bat)):
        infos = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            infos = fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / reps
        out[name] = {"ms": round(ms, 3), "solves_per_s": round(1000.0 * k / ms, 1),
                     "iters": [i.iters for i in infos],
                     "max_relres": max(i.relres for i in infos)}
    vs = [torch.randn(2 * n * M * M, dtype=torch.float64, device="cuda") for _ in range(k)]
    ws = [torch.empty_like(v) for v in vs]
    for name, fn in (("pc_sequential_ms", lambda: [pl.pc_apply(v, w) for pl, v, w in zip(plans, vs, ws)]),
                     ("pc_batch_ms", lambda: batch.pc_apply(vs, ws))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            fn()
        torch.cuda.synchronize()
        out[name] = round((time.perf_counter() - t0) * 1000.0 / 20, 4)
    out["speedup"] = round(out["sequential"]["ms"] / out["batch"]["ms"], 3)
    batch.close()
    for pl in plans:
        pl.close()
    log(f"batch: {out}")
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCE = {"tfft": "wc_pc.hip", "dst": "wc_pc.hip", "pair": "wc_pc.hip", "mg": "wc_mg.hip"}


def measured_traffic(kernel, workload, args):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    profiles/<kernel>_<workload>_pmc.md (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy),
    or None when there is none for this configuration or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path) or args.precision != "fp64" or args.method != "gmres_ps":
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    # the kernel's source file and the shared header (launch constants live there)
    digest = hashlib.sha256()
    for src in (KERNEL_SOURCE.get(kernel.split("_")[0], "wc_ops.hip"), "wc_internal.h"):
        with open(os.path.join(ROOT, "paper_2406_00952_amd", "csrc", src), "rb") as fh:
            digest.update(fh.read())
    digest = digest.hexdigest()
    if fields.get("source_sha256") != digest or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(args, d, gpu_iters):
    """Oracle timed on this host: setup + rhs + `cpu_iters` Krylov iterations on the
    full-size problem, scaled linearly to the GPU's iteration count."""
    import numpy as np
    from oracle.discretization import Problem, AllAtOnce, rhs_tilde, transformed_rhs
    from oracle.precond import FastPreconditioner
    from oracle import krylov, solver as osolver
    kind, symmetric = osolver.METHODS[args.method]
    pr = Problem(dims=args.dims, M=args.M, n=args.n, theta=args.theta, gamma=args.gamma,
                 a_face=d.get("a_face"))
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


SERVE_SHAPES = [(2, 63, 64), (2, 127, 128), (2, 255, 256), (1, 255, 256), (1, 511, 512)]
SERVE_WEIGHTS = [0.3, 0.3, 0.15, 0.15, 0.1]


def serve(args):
    """Poisson arrivals of a mixed population (grid and steps from SERVE_SHAPES, theta in
    {1, 1/2}, gamma = 10^U(-6,-2), a = 1 or the sinusoidal coefficient on grids up to
    M = 127, FP64 or mixed precision 50/50, GMRES-P_S; with --lowrank the a = 1 requests use
    the low-rank form, FP32 ones in 2D only), served by the library's server.
    Reports p50/p99 of submission-to-completion latency and completed solves/s per
    arrival rate, with the latency of each request class run alone for reference."""
    import numpy as np
    import torch
    import datagen
    from paper_2406_00952_amd import wc

    rng = np.random.default_rng(args.seed)
    pool = {}
    for (dims, M, n) in SERVE_SHAPES:
        d = datagen.config_problem(dims, M, n, seed=args.seed, noise_sigma=1e-3)
        pool[(dims, M, n)] = tuple(torch.from_numpy(d[k]).to("cuda") for k in ("f", "g", "y0"))
    torch.cuda.synchronize()

    def draw():
        dims, M, n = SERVE_SHAPES[rng.choice(len(SERVE_SHAPES), p=SERVE_WEIGHTS)]
        coeff = "sin" if (M <= 127 and rng.random() < 0.5) else "const"
        precision = str(rng.choice(["fp64", "mixed"]))
        lowrank = bool(args.lowrank) and coeff == "const" and (dims == 2 or precision == "fp64")
        return dict(dims=dims, M=M, n=n, theta=float(rng.choice([1.0, 0.5])),
                    gamma=float(10.0 ** rng.uniform(-6, -2)),
                    a_face=datagen.sinusoidal_a(dims, M) if coeff == "sin" else None,
                    precision=precision, method="gmres_ps", lowrank=lowrank)

    srv = wc.Server(hbm_budget=0, max_concurrency=args.concurrency)
    # warm the plan cache-free path once per shape (first-use costs out of the timed runs)
    for (dims, M, n) in SERVE_SHAPES:
        f, g, y0 = pool[(dims, M, n)]
        y = torch.empty(n * M ** dims, dtype=torch.float64, device="cuda")
        t = srv.submit(f, g, y0, y, torch.empty_like(y), dims=dims, M=M, n=n, theta=0.5,
                       lowrank=bool(args.lowrank))
        srv.wait(t)
    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        reqs = [draw() for _ in range(args.requests)]
        gaps = rng.exponential(1.0 / rate, size=len(reqs))
        outs, tickets = [], []
        t0 = time.perf_counter()
        due = t0
        for kw, gap in zip(reqs, gaps):
            due += gap
            while time.perf_counter() < due:
                time.sleep(min(0.0005, max(0.0, due - time.perf_counter())))
            f, g, y0 = pool[(kw["dims"], kw["M"], kw["n"])]
            y = torch.empty(kw["n"] * kw["M"] ** kw["dims"], dtype=torch.float64, device="cuda")
            p = torch.empty_like(y)
            outs.append((y, p))
            tickets.append(srv.submit(f, g, y0, y, p, **kw))
        lat, qs, bad = [], [], 0
        for t in tickets:
            info, q_ms, tot_ms = srv.wait(t)
            lat.append(tot_ms)
            qs.append(q_ms)
            bad += int(info.status != wc.WC_OK or info.relres > 1e-8)
        t1 = time.perf_counter()
        lat = np.array(lat)
        results.append({"rate": rate, "requests": len(reqs), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                        "p99_ms": round(float(np.percentile(lat, 99)), 2),
                        "queue_p50_ms": round(float(np.percentile(qs, 50)), 2),
                        "solves_per_s": round(len(reqs) / (t1 - t0), 2), "failed": bad})
        log(f"rate {rate}: {results[-1]}")
        del outs
    srv.close()
    print(json.dumps({"metric": "served latency p50/p99 (ms) and solves/s", "n_gpus": 1,
                      "concurrency": args.concurrency, "data": "synthetic",
                      "population": {"shapes": SERVE_SHAPES, "weights": SERVE_WEIGHTS,
                                     "method": "gmres_ps", "tol": 1e-8,
                                     "lowrank": bool(args.lowrank)},
                      "rates": results}), flush=True)


def main():
    args = parse()
    if (args.method != "gmres_ps" or args.coeff != "const"
            or (args.precision != "fp64" and args.dims != 2)):
        args.lowrank = 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the solver runs on "
              "a single GPU", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    import numpy as np
    import torch
    import datagen
    from paper_2406_00952_amd import wc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    d = datagen.config_problem(args.dims, args.M, args.n, seed=args.seed, noise_sigma=1e-3)
    d["a_face"] = datagen.sinusoidal_a(args.dims, args.M) if args.coeff == "sin" else None
    m = args.M ** args.dims
    n = args.n
    f = torch.from_numpy(d["f"]).to(dev)
    g = torch.from_numpy(d["g"]).to(dev)
    y0 = torch.from_numpy(d["y0"]).to(dev)
    y = torch.empty(n * m, dtype=torch.float64, device=dev)
    p = torch.empty_like(y)
    plan = wc.Plan(args.dims, args.M, n, theta=args.theta, gamma=args.gamma, method=args.method,
                   precision=args.precision, restart=args.restart, tol=1e-8, maxit=500,
                   a_face=d["a_face"], flexible=bool(args.flexible) and not args.lowrank,
                   graphs=bool(args.graphs), lowrank=bool(args.lowrank),
                   mg_tol=args.mg_tol, mg_max_cycles=args.mg_cycles)
    log(f"plan footprint {plan.footprint / 2**30:.2f} GiB")
    tiles = plan.autotune(reps=3) if args.autotune else (0, 0)
    log(f"tile widths (time FFT, x2 pass): {tiles}")
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
    # the same solves without the per-kernel events (captured iterations replayed when
    # graphs are on): the production rate; `value` stays the traced figure above
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    for i in range(args.steps):
        plan.solve(f, g, y0, y, p)
    torch.cuda.synchronize()
    untraced_ms = (time.perf_counter() - u0) * 1000.0 / args.steps
    log(f"untraced: {untraced_ms:.3f} ms per solve")

    # ---- the standard form of the same solve (full-length basis, matvec each step) -----
    standard = None
    if args.lowrank and args.standard_steps > 0:
        sp = wc.Plan(args.dims, args.M, n, theta=args.theta, gamma=args.gamma,
                     method=args.method, precision=args.precision, restart=args.restart,
                     tol=1e-8, maxit=500, a_face=d["a_face"], flexible=bool(args.flexible),
                     graphs=bool(args.graphs))
        if args.autotune:
            sp.autotune(reps=3)
        sp.solve(f, g, y0, y, p)
        torch.cuda.synchronize()
        ts0 = time.perf_counter()
        for _ in range(args.standard_steps):
            si = sp.solve(f, g, y0, y, p)
        torch.cuda.synchronize()
        standard = {"ms_per_solve": round((time.perf_counter() - ts0) * 1000.0 / args.standard_steps, 3),
                    "iters": si.iters, "relres": si.relres, "steps": args.standard_steps,
                    "flexible": bool(args.flexible)}
        log(f"standard form: {standard}")
        sp.close()
        del sp
        torch.cuda.empty_cache()

    batch = batch_bench(args) if args.batch > 0 else None

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
    if args.coeff == "sin":  # the multigrid apply has no fixed pass count
        pc_bytes = None
    pc_gbs = pc_bytes / (pc_ms * 1e-3) / 1e9 if pc_bytes else None

    # ---- plain copy of one system vector: the practical HBM ceiling, and the kernel
    #      that calibrates the FETCH_SIZE / WRITE_SIZE counters (known bytes per dispatch)
    src = torch.randn(2 * n * m, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / 10
    copy_bytes = 2 * src.numel() * 8
    del src, dst

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

    workload = (f"heat{args.dims}d{'_sin' if args.coeff == 'sin' else ''}_M{args.M}_n{args.n}")
    traffic = measured_traffic(dom, workload, args)
    out = {
        "metric": "solve ms to 1e-8 rel. residual; PC-apply HBM GB/s; p50/p99 served latency",
        "value": round(ms_per_step, 3),
        "unit": "ms per solve",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64 Krylov / f32 preconditioner",
        "data": "synthetic",
        "config": {"workload": workload,
                   "coeff": args.coeff,
                   "dims": args.dims, "M": args.M, "n": n, "theta": args.theta,
                   "gamma": args.gamma, "zeta": "pi", "method": args.method,
                   "precision": args.precision, "restart": args.restart, "tol": 1e-8,
                   "flexible": bool(args.flexible) and not args.lowrank,
                   "lowrank": bool(args.lowrank), "tiles_ts_tx": list(tiles),
                   "mg_tol": args.mg_tol if args.coeff == "sin" else None,
                   "mg_cycles": args.mg_cycles if args.coeff == "sin" else None,
                   "dof": 2 * n * m, "seed": args.seed},
        "iters": iters, "relres": relres, "reorth": infos[-1].reorth,
        "untraced_ms_per_solve": round(untraced_ms, 3),
        "mg_cycles_max": infos[-1].mg_cycles_max,
        "solves_per_s": round(1000.0 / ms_per_step, 3),
        "standard_form": standard,
        "batch": batch,
        "pc_apply": {"ms": round(pc_ms, 4), "model_bytes": pc_bytes,
                     "GBps": round(pc_gbs, 1) if pc_gbs else None,
                     "frac_of_peak": round(pc_gbs / HBM_PEAK_GBS, 4) if pc_gbs else None,
                     "kernels": pc_kernels},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "avg_us": round(tot_ms * 1000.0 / launches, 2),
                     "bytes_per_launch": tot_bytes / launches},
        "kernels": kernels,
        "copy": {"bytes": copy_bytes, "ms": round(copy_ms, 4),
                 "GBps": round(copy_bytes / (copy_ms * 1e-3) / 1e9, 1)},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args, d, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
