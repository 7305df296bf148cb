"""GPU parity: every building block and the whole solve through the C ABI against
the CPU FP64 oracle, on the same seeded inputs.

Tolerances: FP64 paths 1e-12 relative (operators) / 1e-10 (solutions at tight
tolerance); the FP32 preconditioner apply 2e-5 relative to max|w| (single
precision transforms of length <= 512 in three directions); solves to the
1e-8 true relative residual with iteration counts within 2 of the oracle.
"""
import numpy as np
import pytest

import datagen
from oracle.discretization import Problem, AllAtOnce, rhs_tilde, transformed_rhs
from oracle.precond import FastPreconditioner
from oracle import solver as osolver

pytestmark = pytest.mark.gpu

KIND = {"gmres_ps": "ps", "minres_abs_ps": "abs_ps", "minres_pms": "pms"}


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_00952_amd import wc
    return torch, wc


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def say(*args):
    print(*args, flush=True)


# ---- operator, rhs, recovery --------------------------------------------------

MV_CASES = [(1, 63, 64, 1.0), (1, 63, 64, 0.5), (2, 31, 16, 0.5), (2, 63, 32, 1.0),
            (2, 15, 8, 0.7), (1, 1000, 5, 0.5), (2, 100, 7, 1.0)]


@pytest.mark.parametrize("dims,M,n,theta", MV_CASES)
@pytest.mark.parametrize("method", ["minres_abs_ps", "gmres_ps", "minres_pms"])
@pytest.mark.parametrize("coeff", ["const", "sin"])
def test_matvec(env, dims, M, n, theta, method, coeff):
    torch, wc = env
    if coeff == "sin" and method == "minres_abs_ps":
        pytest.skip("|P_S| is defined for a = 1 only")
    a_face = None if coeff == "const" else datagen.sinusoidal_a(dims, M)
    say("matvec", dims, M, n, theta, method, coeff)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=1e-3, a_face=a_face)
    plan = wc.Plan(dims, M, n, theta=theta, gamma=1e-3, a_face=a_face, method=method)
    x = datagen.random_vector(1, 2 * n * pr.m)
    xd = dev(torch, x)
    yd = torch.empty_like(xd)
    plan.matvec(xd, yd)
    torch.cuda.synchronize()
    op = AllAtOnce(pr)
    ref = op.A(x) if method != "gmres_ps" else op.Ahat(x)
    assert relerr(host(yd), ref) < 1e-12


@pytest.mark.parametrize("dims,M,n,theta", [(1, 63, 64, 1.0), (2, 31, 16, 0.5), (2, 20, 9, 0.6)])
@pytest.mark.parametrize("method", ["minres_abs_ps", "gmres_ps"])
@pytest.mark.parametrize("coeff", ["const", "sin"])
def test_rhs_and_recover(env, dims, M, n, theta, method, coeff):
    torch, wc = env
    if coeff == "sin" and method == "minres_abs_ps":
        pytest.skip("|P_S| is defined for a = 1 only")
    a_face = None if coeff == "const" else datagen.sinusoidal_a(dims, M)
    say("rhs/recover", dims, M, n, theta, method, coeff)
    gamma = 1e-3
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=gamma, a_face=a_face)
    d = datagen.config_problem(dims, M, n, seed=4, noise_sigma=1e-3)
    y0 = datagen.smooth_modes(9, dims, M, 1, 1.0)[0]
    plan = wc.Plan(dims, M, n, theta=theta, gamma=gamma, a_face=a_face, method=method)
    b = torch.empty(2 * n * pr.m, dtype=torch.float64, device="cuda")
    plan.rhs(dev(torch, d["f"]), dev(torch, d["g"]), dev(torch, y0), b)
    gt, ft = rhs_tilde(pr, d["f"], d["g"], y0)
    ref = transformed_rhs(pr, gt, ft, method != "gmres_ps")
    torch.cuda.synchronize()
    assert relerr(host(b), ref) < 1e-13
    x = datagen.random_vector(2, 2 * n * pr.m)
    y = torch.empty(n * pr.m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    u = torch.empty_like(y)
    plan.recover(dev(torch, x), y, p, u)
    ry, rp, ru = osolver.recover(pr, x)
    torch.cuda.synchronize()
    assert relerr(host(y).reshape(n, -1), ry) < 1e-12
    assert relerr(host(p).reshape(n, -1), rp) < 1e-12
    assert relerr(host(u).reshape(n, -1), ru) < 1e-12


# ---- preconditioner -----------------------------------------------------------

PC_CASES = [(1, 63, 64, 1.0), (1, 63, 64, 0.5), (1, 255, 16, 0.5), (1, 7, 4, 1.0),
            (2, 31, 16, 0.5), (2, 63, 32, 1.0), (2, 15, 8, 0.5), (2, 127, 8, 0.5),
            (2, 7, 128, 1.0), (2, 3, 4, 0.5)]


@pytest.mark.parametrize("dims,M,n,theta", PC_CASES)
@pytest.mark.parametrize("method", ["gmres_ps", "minres_abs_ps", "minres_pms"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pc_apply(env, dims, M, n, theta, method, precision):
    torch, wc = env
    say("pc", dims, M, n, theta, method, precision)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=1e-4)
    plan = wc.Plan(dims, M, n, theta=theta, gamma=1e-4, method=method, precision=precision)
    v = datagen.random_vector(3, 2 * n * pr.m)
    vd = dev(torch, v)
    wd = torch.empty_like(vd)
    plan.pc_apply(vd, wd)
    ref = FastPreconditioner(pr, KIND[method]).apply(v)
    torch.cuda.synchronize()
    err = relerr(host(wd), ref)
    assert err < (1e-12 if precision == "fp64" else 2e-5), err
    # in place
    plan.pc_apply(vd, vd)
    torch.cuda.synchronize()
    assert relerr(host(vd), ref) < (1e-12 if precision == "fp64" else 2e-5)


def test_pc_apply_full_size_fp64(env):
    """2D, M = 255, n = 256 (the 2D Crank-Nicolson workload's size), all outputs."""
    torch, wc = env
    dims, M, n = 2, 255, 256
    say("pc full size", dims, M, n)
    pr = Problem(dims=dims, M=M, n=n, theta=0.5, gamma=1e-4)
    plan = wc.Plan(dims, M, n, theta=0.5, gamma=1e-4, method="gmres_ps")
    v = datagen.random_vector(5, 2 * n * pr.m)
    vd = dev(torch, v)
    wd = torch.empty_like(vd)
    plan.pc_apply(vd, wd)
    ref = FastPreconditioner(pr, "ps").apply(v)
    torch.cuda.synchronize()
    assert relerr(host(wd), ref) < 1e-12


def test_matvec_full_size(env):
    torch, wc = env
    dims, M, n = 2, 255, 256
    say("matvec full size", dims, M, n)
    pr = Problem(dims=dims, M=M, n=n, theta=0.5, gamma=1e-4)
    plan = wc.Plan(dims, M, n, theta=0.5, gamma=1e-4, method="gmres_ps")
    x = datagen.random_vector(6, 2 * n * pr.m)
    xd = dev(torch, x)
    yd = torch.empty_like(xd)
    plan.matvec(xd, yd)
    ref = AllAtOnce(pr).Ahat(x)
    torch.cuda.synchronize()
    assert relerr(host(yd), ref) < 1e-12


# ---- whole solve -------------------------------------------------------------

SOLVE_CASES = [
    # dims, M, n, theta, gamma, method
    (1, 63, 64, 1.0, 1e-4, "minres_abs_ps"),
    (1, 63, 64, 1.0, 1e-4, "gmres_ps"),
    (1, 63, 64, 0.5, 1e-2, "minres_pms"),
    (2, 31, 32, 0.5, 1e-4, "gmres_ps"),
    (2, 31, 32, 0.5, 1e-6, "minres_abs_ps"),
    (2, 15, 16, 1.0, 1e-2, "minres_pms"),
    (2, 63, 64, 0.5, 1e-2, "gmres_ps"),
]


@pytest.mark.parametrize("dims,M,n,theta,gamma,method", SOLVE_CASES)
def test_solve_matches_oracle(env, dims, M, n, theta, gamma, method):
    torch, wc = env
    say("solve", dims, M, n, theta, gamma, method)
    d = datagen.config_problem(dims, M, n, seed=0, noise_sigma=1e-3)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=gamma)
    ref = osolver.solve(pr, d["f"], d["g"], d["y0"], method, tol=1e-8)
    plan = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method=method, tol=1e-8)
    f, g, y0 = dev(torch, d["f"]), dev(torch, d["g"]), dev(torch, d["y0"])
    y = torch.empty(n * pr.m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    info = plan.solve(f, g, y0, y, p)
    say("  gpu iters", info.iters, "relres", info.relres, "oracle iters", ref["iters"])
    assert info.relres <= 1e-8
    assert abs(info.iters - ref["iters"]) <= 2
    # independent FP64 check of the GPU solution's residual with the oracle operator
    x = torch.empty(2 * n * pr.m, dtype=torch.float64, device="cuda")
    b = torch.empty_like(x)
    plan.rhs(f, g, y0, b)
    plan.krylov(b, x)
    xh = host(x)
    op = AllAtOnce(pr)
    A = op.A if method != "gmres_ps" else op.Ahat
    res = np.linalg.norm(ref["b"] - A(xh)) / np.linalg.norm(ref["b"])
    assert res <= 1.05e-8
    # tight tolerance: both sides converge to rounding level and agree
    ref_t = osolver.solve(pr, d["f"], d["g"], d["y0"], method, tol=1e-13, maxit=400)
    plan_t = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method=method, tol=1e-13, maxit=400)
    info_t = plan_t.solve(f, g, y0, y, p)
    sc = max(np.abs(ref_t["y"]).max(), np.abs(ref_t["p"]).max())
    assert np.abs(host(y).reshape(n, -1) - ref_t["y"]).max() <= 1e-10 * sc
    assert np.abs(host(p).reshape(n, -1) - ref_t["p"]).max() <= 1e-10 * sc


@pytest.mark.parametrize("method", ["gmres_ps", "minres_abs_ps"])
def test_mixed_precision_solve(env, method):
    torch, wc = env
    dims, M, n, theta, gamma = 2, 63, 64, 0.5, 1e-4
    say("mixed solve", method)
    d = datagen.config_problem(dims, M, n, seed=1, noise_sigma=1e-3)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=gamma)
    ref = osolver.solve(pr, d["f"], d["g"], d["y0"], method, tol=1e-12, maxit=400)
    plan = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method=method, precision="mixed",
                   tol=1e-8, maxit=400)
    y = torch.empty(n * pr.m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    info = plan.solve(dev(torch, d["f"]), dev(torch, d["g"]), dev(torch, d["y0"]), y, p)
    say("  mixed iters", info.iters, "restarts", info.restarts, "relres", info.relres)
    assert info.relres <= 1e-8
    sc = max(np.abs(ref["y"]).max(), np.abs(ref["p"]).max())
    err = max(np.abs(host(y).reshape(n, -1) - ref["y"]).max(),
              np.abs(host(p).reshape(n, -1) - ref["p"]).max()) / sc
    say("  error vs FP64 oracle", err)
    assert err < 1e-5


@pytest.mark.parametrize("hexp", [5, 6, 7])
@pytest.mark.parametrize("gamma", [1e-10, 1e-6, 1e-2])
def test_table1_example1_gpu(env, hexp, gamma):
    """Table 1 of the paper (Example 1, CN, zeta = pi): GMRES-P_S iterations and e_h."""
    torch, wc = env
    from conftest import load_golden
    row = [r for r in load_golden("table1_example1_cn.txt")
           if int(r[1]) == hexp and float(r[0]) == gamma][0]
    M, n = 2 ** hexp - 1, 2 ** hexp
    say("table1", hexp, gamma)
    d = datagen.example1(M, n)
    pr = Problem(dims=2, M=M, n=n, theta=0.5, gamma=gamma)
    plan = wc.Plan(2, M, n, theta=0.5, gamma=gamma, method="gmres_ps")
    y = torch.empty(n * pr.m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    info = plan.solve(dev(torch, d["f"]), dev(torch, d["g"]), dev(torch, d["y0"]), y, p)
    eh = osolver.e_h(pr, host(y).reshape(n, -1), host(p).reshape(n, -1), d["y_exact"], d["p_exact"])
    say("  iters", info.iters, "e_h", eh)
    assert info.iters == int(row[3])
    assert float(f"{eh:.3g}") == pytest.approx(float(row[4]), rel=1e-9)


@pytest.mark.parametrize("lowrank", [False, True])
@pytest.mark.parametrize("graphs", [False, True])
def test_second_gram_schmidt_pass(env, lowrank, graphs):
    """1D M=63, n=64 at tol 1e-12 takes the second (DGKS) Gram-Schmidt pass, which the host
    launches after reading the flag; the solve must still match the oracle's."""
    torch, wc = env
    dims, M, n, theta, gamma = 1, 63, 64, 0.5, 1e-4
    say("second GS pass, lowrank", lowrank, "graphs", graphs)
    d = datagen.config_problem(dims, M, n, seed=3, noise_sigma=1e-3)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=gamma)
    ref = osolver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-13, maxit=400)
    plan = wc.Plan(dims, M, n, theta=theta, gamma=gamma, method="gmres_ps", tol=1e-12,
                   maxit=400, lowrank=lowrank, graphs=graphs)
    y = torch.empty(n * pr.m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    info = plan.solve(dev(torch, d["f"]), dev(torch, d["g"]), dev(torch, d["y0"]), y, p)
    say("  iters", info.iters, "reorth", info.reorth, "relres", info.relres)
    assert info.reorth >= 1  # the case exercises the second pass
    assert info.relres <= 1e-12
    sc = max(np.abs(ref["y"]).max(), np.abs(ref["p"]).max())
    assert np.abs(host(y).reshape(n, -1) - ref["y"]).max() <= 1e-10 * sc
    assert np.abs(host(p).reshape(n, -1) - ref["p"]).max() <= 1e-10 * sc
