"""Benchmark: whole optimal-control solves on one MI355X.

One step = one complete solve of the workload (right-hand side assembly, the
preconditioned Krylov solve to a 1e-8 true relative residual, recovery of y
and p), inputs resident in HBM.  Prints one JSON line.

Default workload (heat2d_M511_n512): 2D heat tracking on the unit square, a = 1,
M = 511 (h = 1/512), n = 512 steps, T = 1, theta = 1/2 (Crank-Nicolson),
gamma = 10^U(-8,-2) drawn for seed 0, seeded smooth modes + N(0, 1e-3) noise in
f and g, zeta = pi; GMRES(30) right-preconditioned with the block
omega-circulant P_S in the standard form: every iteration runs the all-at-once
matvec and the three-step preconditioner apply (time FFT, sine transforms with
the per-mode 2x2 solves, inverse transforms), FP64 throughout.  `value` is that
solve's time.

Also measured in the same run (extra keys of the same line):
  * per-kernel HIP-event timings over the timed region (library tracing); the
    roofline entry is the preconditioner-apply kernel family with the largest
    share of time, achieved = algorithmic bytes per launch / average duration;
  * the preconditioner apply alone (five passes, 160 nm bytes FP64);
  * mixed precision: the same solve with the FP32 preconditioner apply (FP64
    Krylov, matvec, inner products and residuals), its speedup over FP64 and
    the difference of its y, p from the FP64 solution;
  * MINRES-|P_S| on the same problem and GMRES-P_S at the gamma draws of seeds 1-3, each
    in FP64 and with the FP32 preconditioner apply (minres_and_gamma_draws);
  * the low-rank form of the GMRES proposition (same iterates, compact basis);
  * the 2D M = 255, n = 256 workload in both forms;
  * a short serving pass (Poisson arrivals of mixed sizes, p50/p99 latency);
  * batches: 8 instances solved in lockstep against one solve after another;
  * zeta_sweep: the workload with omega = e^{i zeta}, zeta in {0.1, 0.01, 0.001} (FFTs
    over all n frequencies: no conjugate symmetry), one FP64 solve and one with the FP32
    preconditioner apply each;
  * next_rows: finite elements (M = 255, n = 256), Neumann data on Table 4's finest
    grid (with its e_h beside the printed value) and a general-size problem
    (M = 300, n = 300), each a timed solve plus its preconditioner apply;
  * cpu_baseline: the CPU oracle on a bounded sample of the same workload
    (setup, right-hand side, one Krylov iteration and recovery on the full-size
    problem, the iteration scaled to the GPU's iteration count).

Usage: python bench.py [--steps K] [--warmup W] [--M 511 --n 512] [--gamma G]
                       [--method gmres_ps|minres_abs_ps|minres_pms] [--serve]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# kernel families of the preconditioner apply (library tracing names)
PC_FAMILIES = ("tfft_fwd", "dst_x1_fwd", "pair_mode", "dst_x1_inv", "tfft_inv", "mg_smooth",
               "mg_restrict", "mg_lds", "mg_norm", "mg_mix")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", type=int, default=2)
    ap.add_argument("--M", type=int, default=511)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--gamma", type=float, default=None,
                    help="default: 10^U(-8,-2) drawn for the seed")
    ap.add_argument("--method", default="gmres_ps")
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick the preconditioner tile widths by timing them first")
    ap.add_argument("--graphs", type=int, default=1,
                    help="replay captured Krylov iterations (not while tracing kernels)")
    ap.add_argument("--flexible", type=int, default=1,
                    help="GMRES stores P^-1 v_j (same iterates; no final preconditioner apply)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mg-tol", type=float, default=1e-10,
                    help="multigrid cycle tolerance (variable a); 0 = exactly --mg-cycles cycles")
    ap.add_argument("--mg-cycles", type=int, default=30, help="multigrid cycle cap (variable a)")
    ap.add_argument("--coeff", choices=["const", "sin"], default="const",
                    help="a = 1, or a = 1 + 0.5 sin(2 pi x1) sin(2 pi x2) (multigrid)")
    ap.add_argument("--pc-reps", type=int, default=10)
    ap.add_argument("--mixed", type=int, default=1, help="also time the FP32-preconditioner solve")
    ap.add_argument("--lowrank-steps", type=int, default=3,
                    help="also time the low-rank form (GMRES-P_S, a = 1); 0 = skip")
    ap.add_argument("--small", type=int, default=1,
                    help="also time the 2D M=255, n=256 workload (standard and low-rank)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=1)
    ap.add_argument("--serve", action="store_true",
                    help="serving mode only: Poisson arrivals of a mixed request population")
    ap.add_argument("--serve-inline", type=int, default=1,
                    help="a short serving pass inside the default run (0 = skip)")
    ap.add_argument("--rates", default="5,20,60,150", help="arrival rates (requests/s), --serve")
    ap.add_argument("--requests", type=int, default=60, help="requests per rate, --serve")
    ap.add_argument("--concurrency", type=int, default=4, help="server workers, --serve")
    ap.add_argument("--zeta-sweep", type=int, default=1,
                    help="also solve the workload with zeta in {0.1, 0.01, 0.001} (full spectrum)")
    ap.add_argument("--minres-gamma", type=int, default=1,
                    help="also solve the workload by MINRES-|P_S| and over the gamma draws of "
                         "seeds 1-3, each in FP64 and with the FP32 preconditioner (2D, a = 1)")
    ap.add_argument("--next-rows", type=int, default=1,
                    help="also time the finite element, Neumann and general-size forms")
    ap.add_argument("--batch", type=int, default=8,
                    help="instances of the small serving shape (2D, M=63, n=64) solved one by "
                         "one and as one batch (0 = skip)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync_ms(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / reps, out


def batch_bench(args):
    """Many instances of small problems: sequential wc_solve (captured iterations) against
    one lockstep batch (one launch per preconditioner pass for all instances of a tile
    shape): `args.batch` instances of 2D M = 63, n = 64, and as many of four uneven shapes
    (M, n) in {63, 127} x {64, 128}."""
    import numpy as np
    import torch
    import datagen
    from paper_2406_00952_amd import wc
    k = args.batch
    shape_sets = {"same": [(63, 64)] * k,
                  "uneven": [[(63, 64), (63, 128), (127, 64), (127, 128)][i % 4]
                             for i in range(k)]}
    out = {"instances": k, "shape": "2D M=63 n=64 fp64 GMRES(30)-P_S",
           "uneven_shapes": shape_sets["uneven"]}
    for label, shapes in shape_sets.items():
        plans = [wc.Plan(2, M, n, theta=0.5, gamma=1e-4, method="gmres_ps", tol=1e-8,
                         maxit=500) for (M, n) in shapes]
        data = []
        for i, (M, n) in enumerate(shapes):
            d = datagen.config_problem(2, M, n, seed=args.seed + 10 + i, noise_sigma=1e-3)
            data.append([torch.from_numpy(np.ascontiguousarray(d[x])).cuda()
                         for x in ("f", "g", "y0")])
        ys = [torch.empty(n * M * M, dtype=torch.float64, device="cuda") for (M, n) in shapes]
        ps = [torch.empty_like(y) for y in ys]
        batch = wc.Batch(plans)
        cols = [[dd[j] for dd in data] for j in range(3)]
        fns = {"sequential": lambda: [pl.solve(*dd, y, p)
                                      for pl, dd, y, p in zip(plans, data, ys, ps)],
               "batch": lambda: batch.solve(cols[0], cols[1], cols[2], ys, ps)}
        res = {}
        for name, fn in fns.items():
            fn()
            ms, infos = sync_ms(torch, fn, 5)
            res[name] = {"ms": round(ms, 3), "solves_per_s": round(1000.0 * k / ms, 1),
                         "iters": [i.iters for i in infos],
                         "max_relres": max(i.relres for i in infos)}
        res["speedup"] = round(res["sequential"]["ms"] / res["batch"]["ms"], 3)
        if label == "same":
            out.update(res)
        else:
            out["uneven"] = res
        batch.close()
        for pl in plans:
            pl.close()
    log(f"batch: {out}")
    return out


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    profiles/<kernel>_<workload>_pmc.md (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy),
    or None when there is none for this configuration or the kernel's source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    digest = hashlib.sha256()
    for src in fields.get("sources", "").split(","):
        src = src.strip()
        if src:
            with open(os.path.join(ROOT, "paper_2406_00952_amd", "csrc", src), "rb") as fh:
                digest.update(fh.read())
    if fields.get("source_sha256") != digest.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def host_cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(args, d, gamma, gpu_iters):
    """Oracle timed on this host: setup + rhs + `cpu_iters` Krylov iterations + recovery on
    the full-size problem, the iterations scaled linearly to the GPU's iteration count."""
    import numpy as np
    from oracle.discretization import Problem, AllAtOnce, rhs_tilde, transformed_rhs
    from oracle.precond import FastPreconditioner
    from oracle import krylov, solver as osolver
    kind, symmetric = osolver.METHODS[args.method]
    pr = Problem(dims=args.dims, M=args.M, n=args.n, theta=args.theta, gamma=gamma,
                 a_face=d.get("a_face"))
    t0 = time.perf_counter()
    op = AllAtOnce(pr)
    gt, ft = rhs_tilde(pr, d["f"], d["g"], d["y0"])
    b = transformed_rhs(pr, gt, ft, symmetric)
    P = FastPreconditioner(pr, kind)
    t1 = time.perf_counter()
    k = max(1, args.cpu_iters)
    if symmetric:
        x, _, _ = krylov.minres(op.A, b, P.apply, tol=1e-30, maxit=k)
    else:
        x, _, _ = krylov.gmres(op.Ahat, b, P.apply, tol=1e-30, restart=args.restart, maxit=k)
    t2 = time.perf_counter()
    osolver.recover(pr, x)
    t3 = time.perf_counter()
    per_iter = (t2 - t1) / k
    est_s = (t1 - t0) + (t3 - t2) + per_iter * max(gpu_iters, 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": round(est_s * 1000.0, 1), "unit": "ms per solve", "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle (NumPy/SciPy FP64) setup+rhs+recovery plus {k} GMRES iteration(s) "
                   f"on the full-size workload ({per_iter:.2f} s per iteration, "
                   f"each a dense O(n^2) time transform, dense sine matrices, the "
                   f"all-at-once operator and the true residual), scaled to the GPU's "
                   f"{gpu_iters} iterations"),
        "host_cpu": host_cpu_model(), "logical_cpus": os.cpu_count(),
        "measured_s": round(t3 - t0, 2),
    }


SERVE_SHAPES = [(2, 63, 64), (2, 127, 128), (2, 255, 256), (2, 511, 512), (1, 255, 256),
                (1, 511, 512)]
SERVE_WEIGHTS = [0.3, 0.25, 0.15, 0.05, 0.15, 0.1]


def serve(args, rates=None, requests=None, quiet=False):
    """Poisson arrivals of a mixed population (grid and steps from SERVE_SHAPES, theta in
    {1, 1/2}, gamma = 10^U(-6,-2), a = 1 or the sinusoidal coefficient on grids up to
    M = 127, FP64 or mixed precision 50/50, GMRES(10)-P_S in the standard form), served by
    the library's server.  Reports p50/p99 of submission-to-completion latency and
    completed solves/s per arrival rate."""
    import numpy as np
    import torch
    import datagen
    from paper_2406_00952_amd import wc

    rates = rates or [float(r) for r in args.rates.split(",")]
    requests = requests or args.requests
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
        return dict(dims=dims, M=M, n=n, theta=float(rng.choice([1.0, 0.5])),
                    gamma=float(10.0 ** rng.uniform(-6, -2)),
                    a_face=datagen.sinusoidal_a(dims, M) if coeff == "sin" else None,
                    precision=precision, method="gmres_ps", restart=10)

    srv = wc.Server(hbm_budget=0, max_concurrency=args.concurrency)
    for (dims, M, n) in SERVE_SHAPES:  # first-use costs out of the timed runs
        f, g, y0 = pool[(dims, M, n)]
        y = torch.empty(n * M ** dims, dtype=torch.float64, device="cuda")
        srv.wait(srv.submit(f, g, y0, y, torch.empty_like(y), dims=dims, M=M, n=n, theta=0.5,
                            restart=10))
    results = []
    for rate in rates:
        reqs = [draw() for _ in range(requests)]
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
        results.append({"rate": rate, "requests": len(reqs),
                        "p50_ms": round(float(np.percentile(lat, 50)), 2),
                        "p99_ms": round(float(np.percentile(lat, 99)), 2),
                        "queue_p50_ms": round(float(np.percentile(qs, 50)), 2),
                        "solves_per_s": round(len(reqs) / (t1 - t0), 2), "failed": bad})
        log(f"serve rate {rate}: {results[-1]}")
        del outs
    srv.close()
    out = {"metric": "served latency p50/p99 (ms) and solves/s", "n_gpus": 1,
           "concurrency": args.concurrency, "data": "synthetic",
           "population": {"shapes": SERVE_SHAPES, "weights": SERVE_WEIGHTS,
                          "method": "gmres_ps", "restart": 10, "tol": 1e-8},
           "rates": results}
    if not quiet:
        print(json.dumps(out), flush=True)
    return out


def time_solve(torch, wc, plan, data, steps, warmup, traced=False):
    """Average ms per solve over `steps` after `warmup` solves (and the kernel statistics of
    the timed solves when traced)."""
    f, g, y0, y, p = data
    for i in range(warmup):
        info = plan.solve(f, g, y0, y, p)
        log(f"  warmup {i}: iters {info.iters} relres {info.relres:.2e} {info.ms:.1f} ms")
    if traced:
        plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for _ in range(steps):
        infos.append(plan.solve(f, g, y0, y, p))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    stats = None
    if traced:
        plan.profile(False)
        stats = plan.profile_read()
    return ms, infos, stats


def pc_apply_bench(torch, plan, nvec, reps):
    """The preconditioner apply alone on a random vector: ms per apply and per-kernel stats."""
    v = torch.randn(nvec, dtype=torch.float64, device="cuda")
    w = torch.empty_like(v)
    for _ in range(3):
        plan.pc_apply(v, w)
    plan.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.pc_apply(v, w)
    e1.record()
    torch.cuda.synchronize()
    plan.profile(False)
    stats = plan.profile_read()
    del v, w
    return e0.elapsed_time(e1) / reps, stats


FP64_VALU_PEAK_TFS = 78.6  # MI355X FP64 vector peak (256 CUs x 4 SIMDs x 2.4 GHz x 32)


def next_rows_bench(torch, wc, dev, steps=3):
    """The forms beyond the headline, each timed on a full solve plus its preconditioner
    apply: finite elements (2D M = 255, n = 256), homogeneous Neumann data on Table 4's
    finest grid (256 nodes per dimension, n = 256, a = 1e-3), and the general path
    (2D M = 300, n = 300: neither size fits the FFT path).  The dense steps of the last two
    are FP64 ALU work; their rate is reported against the FP64 vector peak."""
    import datagen
    res = {}

    def run(name, plan, data, nvec, dense_flops=None, extra=None):
        if args_autotune[0]:
            plan.autotune(reps=2)
        ms, infos, _ = time_solve(torch, wc, plan, data, steps, 1)
        pc_ms, st = pc_apply_bench(torch, plan, nvec, 5)
        r = {"ms_per_solve": round(ms, 3), "iters": infos[-1].iters,
             "relres": max(i.relres for i in infos), "pc_apply_ms": round(pc_ms, 4)}
        if dense_flops:
            dense_ms = sum(v[1] for k, v in st.items() if k in ("dst_x1_fwd", "dst_x1_inv")) / 5
            r["dense_spatial_ms"] = round(dense_ms, 4)
            r["dense_spatial_TFLOPs"] = round(dense_flops / (dense_ms * 1e-3) / 1e12, 2)
            r["dense_frac_of_fp64_peak"] = round(dense_flops / (dense_ms * 1e-3) / 1e12 /
                                                 FP64_VALU_PEAK_TFS, 4)
        if extra:
            r.update(extra())
        res[name] = r
        log(f"{name}: {r}")
        plan.close()

    def tens(dd, n, m):
        t = [torch.from_numpy(np.ascontiguousarray(dd[k])).to(dev) for k in ("f", "g", "y0")]
        y = torch.empty(n * m, dtype=torch.float64, device=dev)
        return (*t, y, torch.empty_like(y))

    import numpy as np
    # finite elements, 2D M = 255, n = 256
    M, n = 255, 256
    dd = datagen.config_problem(2, M, n, seed=3, noise_sigma=1e-3)
    data = tens(dd, n, M * M)
    run("fem_heat2d_M255_n256", wc.Plan(2, M, n, theta=0.5, gamma=1e-4, method="gmres_ps",
                                        tol=1e-8, disc="fem"), data, 2 * n * M * M)
    # Neumann data, Example 3 at h = 2^-8: 256 nodes per dimension, n = 256
    N = 256
    dd = datagen.example3(N, N)
    data = tens(dd, N, N * N)
    lines = N * N  # lines of one dense x1 pass: n slabs x N rows
    flops = 4 * (4.0 * lines * N * N)  # four dense passes, 4 flops per complex-real term

    def eh():  # the error of Section 4: max over the 2n time slices of h ||slice error||_2
        yy = data[3].cpu().numpy().reshape(N, -1)
        pp = data[4].cpu().numpy().reshape(N, -1)
        ey = np.linalg.norm(yy - dd["y_exact"][1:], axis=1).max()
        ep = np.linalg.norm(pp - dd["p_exact"][:-1], axis=1).max()
        return {"e_h": float(max(ey, ep) / (N - 1)), "e_h_printed": 5.10e-9}
    run("neumann_example3_N256_n256", wc.Plan(2, N, N, theta=0.5, gamma=1e-4, method="gmres_ps",
                                              tol=1e-8, bc="neumann", kappa=1e-3),
        data, 2 * N * N * N, flops, eh)
    # general path, 2D M = 300, n = 300
    M, n = 300, 300
    dd = datagen.config_problem(2, M, n, seed=4, noise_sigma=1e-3)
    data = tens(dd, n, M * M)
    flops = 4 * (4.0 * 2 * n * M * M * M)  # 2n slabs of M lines
    run("general_heat2d_M300_n300", wc.Plan(2, M, n, theta=0.5, gamma=1e-4, method="gmres_ps",
                                            tol=1e-8), data, 2 * n * M * M, flops)
    torch.cuda.empty_cache()
    return res


def zeta_sweep_bench(torch, wc, data, common, M, n):
    """The mixed-precision workload's omega = e^{i zeta}, zeta in {0.1, 0.01, 0.001}, on the
    same 2D M = 511, n = 512 problem: zeta != pi, so each block row's spectrum has no
    conjugate symmetry and all n frequencies are transformed (n-point FFTs, the transposed
    sine passes over 2n slabs).  One FP64 solve each (at most 200 iterations), then one with
    the FP32 preconditioner apply (at most 100 iterations; near omega = 1 it may stop there,
    reported with its residual) and the largest difference of its y, p from the FP64
    solution."""
    y, p = data[3], data[4]
    res = {}
    for zeta in (0.1, 0.01, 0.001):
        plan = wc.Plan(2, M, n, precision="fp64", flexible=True, zeta=zeta,
                       **dict(common, maxit=200))
        ms, infos, _ = time_solve(torch, wc, plan, data, 1, 0)
        r = {"ms_per_solve": round(ms, 1), "iters": infos[-1].iters, "relres": infos[-1].relres}
        plan.close()
        torch.cuda.empty_cache()
        yr, pr = y.clone(), p.clone()
        mp = wc.Plan(2, M, n, precision="mixed", flexible=True, zeta=zeta,
                     **dict(common, maxit=100))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf = mp.solve(*data, allow_maxit=True)
        torch.cuda.synchronize()
        sc = max(float(yr.abs().max()), float(pr.abs().max()))
        r["mixed"] = {"ms_per_solve": round((time.perf_counter() - t0) * 1000.0, 1),
                      "iters": inf.iters, "relres": inf.relres,
                      "converged": bool(inf.status == wc.WC_OK),
                      "max_rel_diff_vs_fp64_solution":
                          max(float((y - yr).abs().max()), float((p - pr).abs().max())) / sc}
        mp.close()
        del yr, pr
        torch.cuda.empty_cache()
        res[str(zeta)] = r
        log(f"zeta {zeta}: {r}")
    return res


def minres_gamma_bench(torch, wc, datagen, args, data, common, y64, p64):
    """The mixed-precision workload's other method and gamma draws: MINRES-|P_S| (zeta = pi)
    and GMRES(30)-P_S with gamma = 10^U(-8,-2) drawn for seeds 1, 2, 3 (the data of the
    headline's seed), each in FP64 and with the FP32 preconditioner apply: iterations,
    ms per solve (one solve after one untimed) and the largest difference of y, p from the
    FP64 standard-form solution of the same problem (MINRES: the headline's)."""
    M, n = args.M, args.n
    y, p = data[3], data[4]
    res = {}

    def solve(plan):
        ms, infos, _ = time_solve(torch, wc, plan, data, 1, 1)
        return {"ms_per_solve": round(ms, 2), "iters": infos[-1].iters,
                "relres": infos[-1].relres}

    def diff(yr, pr):
        sc = max(float(yr.abs().max()), float(pr.abs().max()))
        return max(float((y - yr).abs().max()), float((p - pr).abs().max())) / sc

    mres = {}
    for prec in ("fp64", "mixed"):
        plan = wc.Plan(2, M, n, precision=prec, **dict(common, method="minres_abs_ps"))
        r = solve(plan)
        r["max_rel_diff_vs_fp64_gmres_solution"] = diff(y64, p64)
        mres[prec] = r
        log(f"minres |P_S| {prec}: {r}")
        plan.close()
        torch.cuda.empty_cache()
    mres["speedup_mixed_vs_fp64"] = round(mres["fp64"]["ms_per_solve"] /
                                          mres["mixed"]["ms_per_solve"], 3)
    res["minres_abs_ps"] = mres
    sweep = {f"seed{seed}": {"gamma": datagen.log_uniform_gamma(seed)} for seed in (1, 2, 3)}
    ref = {}
    for prec in ("fp64", "mixed"):  # one plan at a time: an FGMRES(30) plan holds 131 GiB
        plan = wc.Plan(2, M, n, precision=prec, flexible=True, **common)
        for key, row in sweep.items():
            plan.retarget(theta=common["theta"], gamma=row["gamma"], tol=common["tol"],
                          maxit=common["maxit"])
            row[prec] = solve(plan)
            if prec == "fp64":
                ref[key] = (y.clone(), p.clone())
            else:
                row[prec]["max_rel_diff_vs_fp64_solution"] = diff(*ref[key])
                row["speedup_mixed_vs_fp64"] = round(row["fp64"]["ms_per_solve"] /
                                                     row["mixed"]["ms_per_solve"], 3)
                log(f"gamma {key}: {row}")
        plan.close()
        torch.cuda.empty_cache()
    del ref
    res["gamma_draws"] = sweep
    return res


args_autotune = [1]


def main():
    args = parse()
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
    gamma = args.gamma if args.gamma is not None else datagen.log_uniform_gamma(args.seed)
    d = datagen.config_problem(args.dims, args.M, args.n, seed=args.seed, noise_sigma=1e-3)
    d["a_face"] = datagen.sinusoidal_a(args.dims, args.M) if args.coeff == "sin" else None
    m = args.M ** args.dims
    n = args.n
    nvec = 2 * n * m
    f = torch.from_numpy(d["f"]).to(dev)
    g = torch.from_numpy(d["g"]).to(dev)
    y0 = torch.from_numpy(d["y0"]).to(dev)
    y = torch.empty(n * m, dtype=torch.float64, device=dev)
    p = torch.empty_like(y)
    data = (f, g, y0, y, p)
    common = dict(theta=args.theta, gamma=gamma, method=args.method, restart=args.restart,
                  tol=1e-8, maxit=500, a_face=d["a_face"], graphs=bool(args.graphs),
                  mg_tol=args.mg_tol, mg_max_cycles=args.mg_cycles)
    workload = f"heat{args.dims}d{'_sin' if args.coeff == 'sin' else ''}_M{args.M}_n{args.n}"

    # ---- headline: FP64, standard form ------------------------------------------------
    plan = wc.Plan(args.dims, args.M, n, precision="fp64", flexible=bool(args.flexible), **common)
    log(f"{workload}: gamma {gamma:.3e}, plan footprint {plan.footprint / 2**30:.2f} GiB")
    tiles = plan.autotune(reps=3) if args.autotune else (0, 0)
    log(f"tile widths (time FFT, x2 pass): {tiles}")
    ms_per_step, infos, stats = time_solve(torch, wc, plan, data, args.steps, args.warmup,
                                           traced=True)
    iters = infos[-1].iters
    relres = max(i.relres for i in infos)
    log(f"fp64 standard: {ms_per_step:.3f} ms, iters {iters}, relres {relres:.2e}")
    untraced_ms, _, _ = time_solve(torch, wc, plan, data, args.steps, 0)
    log(f"  untraced: {untraced_ms:.3f} ms per solve")
    y64 = y.clone()
    p64 = p.clone()
    pc_ms, pc_stats = pc_apply_bench(torch, plan, nvec, args.pc_reps)
    plan.close()
    del plan
    torch.cuda.empty_cache()

    es = 16  # FP64 complex
    if args.coeff == "const":
        passes = 5 if args.dims == 2 else 3
        pc_bytes = passes * 2 * nvec * 8  # 160 nm B (2D) / 96 nm B (1D)
    else:
        pc_bytes = None  # the multigrid apply has no fixed pass count
    pc_gbs = pc_bytes / (pc_ms * 1e-3) / 1e9 if pc_bytes else None

    # ---- mixed precision: FP32 preconditioner apply, FP64 everything else --------------
    mixed = None
    if args.mixed:
        mp = wc.Plan(args.dims, args.M, n, precision="mixed", flexible=True, **common)
        if args.autotune:
            mp.autotune(reps=3)
        mms, minf, _ = time_solve(torch, wc, mp, data, args.steps, 1)
        mpc_ms, _ = pc_apply_bench(torch, mp, nvec, args.pc_reps)
        sc = max(float(y64.abs().max()), float(p64.abs().max()))
        diff = max(float((y - y64).abs().max()), float((p - p64).abs().max())) / sc
        mixed = {"ms_per_solve": round(mms, 3), "iters": minf[-1].iters,
                 "relres": max(i.relres for i in minf),
                 "speedup_vs_fp64": round(untraced_ms / mms, 3),
                 "max_rel_diff_vs_fp64_solution": diff,
                 "pc_apply_ms": round(mpc_ms, 4),
                 "pc_apply_model_bytes": 6 * nvec * 8 if args.dims == 2 else None,
                 "dtype": "f64 Krylov / f32 preconditioner apply"}
        log(f"mixed: {mixed}")
        mp.close()
        del mp
        torch.cuda.empty_cache()

    # ---- MINRES-|P_S| and the other gamma draws, FP64 and mixed -------------------------
    mg = None
    if (args.minres_gamma and args.dims == 2 and args.coeff == "const"
            and args.method == "gmres_ps"):
        mg = minres_gamma_bench(torch, wc, datagen, args, data, common, y64, p64)

    # ---- low-rank form (same iterates, compact Krylov basis) ---------------------------
    lowrank = None
    if args.lowrank_steps > 0 and args.method == "gmres_ps" and args.coeff == "const":
        lp = wc.Plan(args.dims, args.M, n, precision="fp64", lowrank=True, **common)
        if args.autotune:
            lp.autotune(reps=3)
        lms, linf, _ = time_solve(torch, wc, lp, data, args.lowrank_steps, 1)
        lowrank = {"ms_per_solve": round(lms, 3), "iters": linf[-1].iters,
                   "relres": max(i.relres for i in linf),
                   "form": "GMRES(30)-P_S Arnoldi in the compact coordinates of the GMRES "
                           "proposition (the preconditioner's time and sine transforms of r0 "
                           "once per cycle)"}
        log(f"lowrank: {lowrank}")
        lp.close()
        del lp
        torch.cuda.empty_cache()

    # ---- the 2D M = 255, n = 256 workload ---------------------------------------------
    small = None
    if args.small and (args.dims, args.M, args.n) != (2, 255, 256) and args.coeff == "const":
        M2, n2 = 255, 256
        d2 = datagen.config_problem(2, M2, n2, seed=args.seed, noise_sigma=1e-3)
        t2 = [torch.from_numpy(d2[k]).to(dev) for k in ("f", "g", "y0")]
        y2 = torch.empty(n2 * M2 * M2, dtype=torch.float64, device=dev)
        data2 = (*t2, y2, torch.empty_like(y2))
        small = {"workload": "heat2d_M255_n256", "gamma": 1e-4, "theta": 0.5}
        for name, kw in (("standard_fp64", dict(flexible=True)), ("lowrank_fp64", dict(lowrank=True)),
                         ("standard_mixed", dict(precision="mixed", flexible=True))):
            c2 = dict(common, gamma=1e-4, a_face=None)
            sp = wc.Plan(2, M2, n2, **dict(c2, **kw))
            if args.autotune:
                sp.autotune(reps=3)
            sms, sinf, _ = time_solve(torch, wc, sp, data2, 5, 1)
            small[name] = {"ms_per_solve": round(sms, 3), "iters": sinf[-1].iters,
                           "relres": max(i.relres for i in sinf)}
            if name == "standard_fp64":
                spc, _ = pc_apply_bench(torch, sp, 2 * n2 * M2 * M2, 20)
                small["pc_apply_ms"] = round(spc, 4)
                small["pc_apply_frac_of_peak"] = round(
                    5 * 2 * 2 * n2 * M2 * M2 * 8 / (spc * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            sp.close()
        log(f"small: {small}")
        torch.cuda.empty_cache()

    batch = batch_bench(args) if args.batch > 0 else None
    args_autotune[0] = args.autotune
    nxt = next_rows_bench(torch, wc, dev) if args.next_rows else None
    zsweep = (zeta_sweep_bench(torch, wc, data, common, args.M, n)
              if args.zeta_sweep and (args.dims, args.M, n, args.coeff) == (2, 511, 512, "const")
              else None)
    served = None
    if args.serve_inline:
        served = serve(args, rates=[10.0, 40.0], requests=30, quiet=True)

    # ---- plain copy of one system vector: the practical HBM ceiling ------------------
    src = torch.randn(nvec, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    copy_ms, _ = sync_ms(torch, lambda: dst.copy_(src), 10)
    copy_bytes = 2 * nvec * 8
    del src, dst

    # ---- roofline: the preconditioner-apply kernel with the largest share of the timed
    #      region; achieved = its algorithmic bytes per launch / its average duration ------
    fam = {k: v for k, v in stats.items() if v[0] > 0}
    pcf = {k: v for k, v in fam.items() if k in PC_FAMILIES}
    dom = max(pcf, key=lambda k: pcf[k][1])
    launches, tot_ms, tot_bytes = pcf[dom]
    achieved = tot_bytes / (tot_ms * 1e-3) / 1e9
    overall = max(fam, key=lambda k: fam[k][1])
    kernels = {k: {"launches": v[0], "avg_us": round(v[1] * 1000.0 / v[0], 2),
                   "share": round(v[1] / sum(x[1] for x in fam.values()), 4),
                   "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1) if v[1] > 0 else None}
               for k, v in sorted(fam.items(), key=lambda kv: -kv[1][1])}
    pc_kernels = {k: {"avg_us": round(v[1] * 1000.0 / v[0], 2),
                      "GBps": round(v[2] / (v[1] * 1e-3) / 1e9, 1)}
                  for k, v in pc_stats.items() if v[0] > 0}
    traffic = measured_traffic(dom, workload, "fp64")
    out = {
        "metric": "solve ms to 1e-8 rel. residual; PC-apply HBM GB/s; p50/p99 served latency",
        "value": round(ms_per_step, 3),
        "unit": "ms per solve",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "coeff": args.coeff,
                   "dims": args.dims, "M": args.M, "n": n, "theta": args.theta,
                   "gamma": gamma, "zeta": "pi", "method": args.method,
                   "form": "standard (matvec and three-step preconditioner apply every "
                           "iteration)",
                   "precision": "fp64", "restart": args.restart, "tol": 1e-8,
                   "flexible": bool(args.flexible), "tiles_ts_tx": list(tiles),
                   "mg_tol": args.mg_tol if args.coeff == "sin" else None,
                   "mg_cycles": args.mg_cycles if args.coeff == "sin" else None,
                   "dof": nvec, "seed": args.seed},
        "iters": iters, "relres": relres, "reorth": infos[-1].reorth,
        "untraced_ms_per_solve": round(untraced_ms, 3),
        "mg_cycles_max": infos[-1].mg_cycles_max,
        "solves_per_s": round(1000.0 / ms_per_step, 3),
        "pc_apply": {"ms": round(pc_ms, 4), "model_bytes": pc_bytes,
                     "GBps": round(pc_gbs, 1) if pc_gbs else None,
                     "frac_of_peak": round(pc_gbs / HBM_PEAK_GBS, 4) if pc_gbs else None,
                     "kernels": pc_kernels},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "avg_us": round(tot_ms * 1000.0 / launches, 2),
                     "bytes_per_launch": tot_bytes / launches,
                     "overall_dominant_kernel": overall},
        "mixed": mixed,
        "minres_and_gamma_draws": mg,
        "lowrank": lowrank,
        "heat2d_M255_n256": small,
        "serve": {"p50_ms": served["rates"][-1]["p50_ms"], "p99_ms": served["rates"][-1]["p99_ms"],
                  "solves_per_s": served["rates"][-1]["solves_per_s"],
                  "rates": served["rates"], "population": served["population"],
                  "concurrency": served["concurrency"]} if served else None,
        "batch": batch,
        "next_rows": nxt,
        "zeta_sweep": zsweep,
        "kernels": kernels,
        "copy": {"bytes": copy_bytes, "ms": round(copy_ms, 4),
                 "GBps": round(copy_bytes / (copy_ms * 1e-3) / 1e9, 1)},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args, d, gamma, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
