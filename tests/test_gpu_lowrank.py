"""GPU parity of the low-rank GMRES form (opts.lowrank): the Arnoldi process in the
compact coordinates given by the GMRES proposition (Ahat - P_S acts only in time, rank
one per block row).  In exact arithmetic its iterates are those of GMRES(k)-P_S, so the
checks are: the oracle's iteration count (within 1), the true residual recomputed with
the oracle's operator, and the solution at a tight tolerance against the oracle's, also
with short restarts (later cycles start from residuals that lie mostly in the
correction's range) and with several block sizes.
"""
import numpy as np
import pytest

import datagen
from oracle.discretization import Problem, AllAtOnce
from oracle import solver as osolver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_00952_amd import wc
    return torch, wc


CASES = [
    # dims, M, n, theta, gamma, restart
    (1, 63, 64, 1.0, 1e-4, 30),
    (1, 255, 16, 0.5, 1e-2, 30),
    (1, 127, 4, 0.7, 1e-6, 30),
    (2, 31, 32, 0.5, 1e-4, 30),
    (2, 63, 64, 0.5, 1e-2, 30),
    (2, 15, 8, 1.0, 1e-8, 30),
    (2, 31, 32, 0.5, 1e-6, 3),   # several restart cycles
    (2, 63, 16, 0.6, 1e-4, 2),
    (2, 127, 4, 1.0, 1e-4, 30),  # two frequencies: most chunks of the contraction are empty
]


@pytest.mark.parametrize("dims,M,n,theta,gamma,restart", CASES)
def test_lowrank_gmres_matches_oracle(env, dims, M, n, theta, gamma, restart):
    torch, wc = env
    print("lowrank", dims, M, n, theta, gamma, restart, flush=True)
    d = datagen.config_problem(dims, M, n, seed=7, noise_sigma=1e-3)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=gamma)
    ref = osolver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-8, restart=restart,
                        maxit=600)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f, g, y0 = dev(d["f"]), dev(d["g"]), dev(d["y0"])
    m = pr.m
    plan = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method="gmres_ps", restart=restart,
                   tol=1e-8, maxit=600, lowrank=True)
    x = torch.empty(2 * n * m, dtype=torch.float64, device="cuda")
    b = torch.empty_like(x)
    plan.rhs(f, g, y0, b)
    info = plan.krylov(b, x)
    print("  gpu iters", info.iters, "restarts", info.restarts, "relres", info.relres,
          "oracle", ref["iters"], flush=True)
    assert info.relres <= 1e-8
    assert abs(info.iters - ref["iters"]) <= 1
    res = np.linalg.norm(ref["b"] - AllAtOnce(pr).Ahat(x.cpu().numpy())) / np.linalg.norm(ref["b"])
    assert res <= 1.05e-8
    # tight tolerance: both converge to rounding level and agree
    ref_t = osolver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-13, restart=restart,
                          maxit=800)
    plan_t = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method="gmres_ps", restart=restart,
                     tol=1e-13, maxit=800, lowrank=True)
    y = torch.empty(n * m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    plan_t.solve(f, g, y0, y, p, allow_maxit=True)
    sc = max(np.abs(ref_t["y"]).max(), np.abs(ref_t["p"]).max())
    assert np.abs(y.cpu().numpy().reshape(n, -1) - ref_t["y"]).max() <= 1e-10 * sc
    assert np.abs(p.cpu().numpy().reshape(n, -1) - ref_t["p"]).max() <= 1e-10 * sc


@pytest.mark.parametrize("M,n", [(255, 256), (511, 16)])
def test_lowrank_full_size_matches_standard(env, M, n):
    """2D, M = 255, n = 256 (the 2D Crank-Nicolson workload), and the 512-point sine
    transforms (M = 511): the low-rank form and the standard form take the same number of
    iterations and reach the same solution."""
    torch, wc = env
    dims = 2
    print("lowrank vs standard", M, n, flush=True)
    d = datagen.config_problem(dims, M, n, seed=0, noise_sigma=1e-3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f, g, y0 = dev(d["f"]), dev(d["g"]), dev(d["y0"])
    out = {}
    for lr in (False, True):
        plan = wc.Plan(dims, M, n, theta=0.5, gamma=1e-4, method="gmres_ps", tol=1e-10,
                       lowrank=lr)
        y = torch.empty(n * M * M, dtype=torch.float64, device="cuda")
        p = torch.empty_like(y)
        info = plan.solve(f, g, y0, y, p)
        out[lr] = (info, y.cpu().numpy(), p.cpu().numpy())
        print("  lowrank", lr, "iters", info.iters, "relres", info.relres, flush=True)
        plan.close()
        del plan
        torch.cuda.empty_cache()
    assert abs(out[True][0].iters - out[False][0].iters) <= 1
    assert out[True][0].relres <= 1e-10
    sc = max(np.abs(out[False][1]).max(), np.abs(out[False][2]).max())
    assert np.abs(out[True][1] - out[False][1]).max() <= 1e-8 * sc
    assert np.abs(out[True][2] - out[False][2]).max() <= 1e-8 * sc


def test_lowrank_rejects_other_methods(env):
    torch, wc = env
    with pytest.raises(wc.WcError):
        wc.Plan(2, 31, 32, method="minres_abs_ps", lowrank=True)
    with pytest.raises(wc.WcError):
        wc.Plan(1, 63, 32, method="gmres_ps", precision="mixed", lowrank=True)  # 2D only


MIXED_CASES = [
    # dims, M, n, theta, gamma, restart
    (2, 31, 32, 0.5, 1e-4, 30),
    (2, 63, 64, 0.5, 1e-2, 30),
    (2, 63, 64, 1.0, 1e-6, 30),
    (2, 31, 32, 0.5, 1e-6, 3),   # several restart cycles
    (2, 127, 16, 0.6, 1e-4, 2),
]


@pytest.mark.parametrize("dims,M,n,theta,gamma,restart", MIXED_CASES)
def test_lowrank_mixed_precision(env, dims, M, n, theta, gamma, restart):
    """Low-rank GMRES with the FP32 preconditioner: the compact Arnoldi process holds
    for the FP32 apply, and the restart on the FP64 true residual removes what FP32
    leaves (each cycle's true residual is at the FP32 level of the last), so the solve
    still meets 1e-8 by the oracle's operator, in at most a few more iterations than the
    oracle's FP64 GMRES, and the solution is within FP32 accuracy of the oracle's."""
    torch, wc = env
    print("lowrank mixed", dims, M, n, theta, gamma, restart, flush=True)
    d = datagen.config_problem(dims, M, n, seed=11, noise_sigma=1e-3)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=gamma)
    ref = osolver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-8, restart=restart,
                        maxit=600)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f, g, y0 = dev(d["f"]), dev(d["g"]), dev(d["y0"])
    plan = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method="gmres_ps", precision="mixed",
                   restart=restart, tol=1e-8, maxit=600, lowrank=True)
    x = torch.empty(2 * n * pr.m, dtype=torch.float64, device="cuda")
    b = torch.empty_like(x)
    plan.rhs(f, g, y0, b)
    info = plan.krylov(b, x)
    res = np.linalg.norm(ref["b"] - AllAtOnce(pr).Ahat(x.cpu().numpy())) / np.linalg.norm(ref["b"])
    print("  gpu iters", info.iters, "restarts", info.restarts, "relres", info.relres,
          "oracle-operator relres", res, "oracle iters", ref["iters"], flush=True)
    assert info.relres <= 1e-8 and res <= 1.05e-8
    assert info.iters <= ref["iters"] + 6
    ref_t = osolver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-12, restart=restart,
                          maxit=800)
    sc = np.abs(ref_t["x"]).max()
    assert np.abs(x.cpu().numpy() - ref_t["x"]).max() <= 1e-5 * sc


def test_full_size_solve_in_bench_configuration(env):
    """The 2D Crank-Nicolson workload (M = 255, n = 256, gamma = 1e-4, seed 0) solved as
    bench.py times it (low-rank GMRES(30)-P_S, autotuned tiles, captured iterations): the
    right-hand side equals the oracle's, the oracle's operator confirms the true relative
    residual, and the iteration count is within 2 of the oracle's own GMRES(30)-P_S."""
    torch, wc = env
    from oracle.discretization import rhs_tilde, transformed_rhs
    dims, M, n = 2, 255, 256
    print("full-size solve", dims, M, n, flush=True)
    d = datagen.config_problem(dims, M, n, seed=0, noise_sigma=1e-3)
    pr = Problem(dims=dims, M=M, n=n, theta=0.5, gamma=1e-4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f, g, y0 = dev(d["f"]), dev(d["g"]), dev(d["y0"])
    plan = wc.Plan(dims, M, n, theta=0.5, gamma=1e-4, method="gmres_ps", tol=1e-8, maxit=500,
                   lowrank=True, graphs=True)
    plan.autotune(reps=2)
    x = torch.empty(2 * n * pr.m, dtype=torch.float64, device="cuda")
    b = torch.empty_like(x)
    plan.rhs(f, g, y0, b)
    for _ in range(2):  # the second solve replays the captured iterations
        info = plan.krylov(b, x)
    xs = x.cpu().numpy()
    gt, ft = rhs_tilde(pr, d["f"], d["g"], d["y0"])
    bref = transformed_rhs(pr, gt, ft, False)
    assert np.abs(b.cpu().numpy() - bref).max() <= 1e-13 * np.abs(bref).max()
    res = np.linalg.norm(bref - AllAtOnce(pr).Ahat(xs)) / np.linalg.norm(bref)
    print("  gpu iters", info.iters, "relres", info.relres, "oracle-operator relres", res,
          flush=True)
    assert info.relres <= 1e-8 and res <= 1.05e-8
    ref = osolver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-8, restart=30)
    print("  oracle iters", ref["iters"], flush=True)
    assert abs(info.iters - ref["iters"]) <= 2
