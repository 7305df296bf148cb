"""GPU tests of the captured Krylov iterations (opts.graphs) and of the tile-width
autotuner: replayed graphs give bitwise the results of eager launches, on every replay,
with eager work and synchronisations between replays; a tuned plan still matches the
oracle."""
import numpy as np
import pytest

import datagen
from oracle.discretization import Problem
from oracle.precond import FastPreconditioner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_00952_amd import wc
    return torch, wc


CASES = [
    # dims, M, n, theta, gamma, method, precision, coeff, extra plan options
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const", {}),
    (2, 31, 32, 1.0, 1e-3, "gmres_ps", "mixed", "const", {}),
    (1, 127, 64, 0.5, 1e-4, "minres_abs_ps", "fp64", "const", {}),
    (2, 31, 32, 0.5, 1e-2, "minres_pms", "fp64", "const", {}),
    (2, 63, 32, 0.5, 1e-4, "gmres_ps", "fp64", "sin", dict(mg_tol=0.0, mg_max_cycles=2)),
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const", dict(lowrank=True, restart=4)),
]


@pytest.mark.parametrize("dims,M,n,theta,gamma,method,precision,coeff,extra", CASES)
def test_graph_replays_match_eager(env, dims, M, n, theta, gamma, method, precision, coeff,
                                   extra):
    torch, wc = env
    print("graphs", dims, M, n, method, precision, coeff, flush=True)
    d = datagen.config_problem(dims, M, n, seed=3, noise_sigma=1e-3)
    a_face = datagen.sinusoidal_a(dims, M) if coeff == "sin" else None
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    f, g, y0 = dev(d["f"]), dev(d["g"]), dev(d["y0"])
    m = M ** dims
    kw = dict(theta=theta, gamma=gamma, method=method, precision=precision, a_face=a_face,
              maxit=400, **extra)
    y_e = torch.empty(n * m, dtype=torch.float64, device="cuda")
    p_e = torch.empty_like(y_e)
    eager = wc.Plan(dims, M, n, graphs=False, **kw)
    ie = eager.solve(f, g, y0, y_e, p_e)
    assert ie.relres <= 1e-8
    ye, pe = y_e.cpu().numpy(), p_e.cpu().numpy()
    plan = wc.Plan(dims, M, n, graphs=True, **kw)
    scratch = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):  # first solve captures, later ones replay
        y = torch.full_like(y_e, float("nan"))
        p = torch.full_like(y_e, float("nan"))
        info = plan.solve(f, g, y0, y, p)
        assert info.iters == ie.iters and info.relres == ie.relres, rep
        assert np.array_equal(y.cpu().numpy(), ye), rep
        assert np.array_equal(p.cpu().numpy(), pe), rep
        scratch.mul_(1.0001).add_(1.0)  # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("dims,M,n,method", [(2, 63, 32, "gmres_ps"), (1, 255, 64, "minres_pms"),
                                             (2, 127, 16, "minres_abs_ps")])
def test_autotune_keeps_parity(env, dims, M, n, method):
    torch, wc = env
    pr = Problem(dims=dims, M=M, n=n, theta=0.5, gamma=1e-4)
    plan = wc.Plan(dims, M, n, theta=0.5, gamma=1e-4, method=method)
    ts, tx = plan.autotune(reps=2)
    print("autotune", dims, M, n, method, "->", ts, tx, flush=True)
    # time passes: packed tiles (> 0) or per-block-row tiles (< 0, n >= 64); x2 pass
    # (2D): column tiles (> 0) or the transposed rows (< 0, M + 1 >= 128)
    assert ts in (4, 8, 16, -8, -16)
    assert tx in ((4, 8, 16, -4, -8) if dims == 2 else (0,))
    v = datagen.random_vector(9, 2 * n * pr.m)
    kind = {"gmres_ps": "ps", "minres_abs_ps": "abs_ps", "minres_pms": "pms"}[method]
    ref = FastPreconditioner(pr, kind).apply(v)
    vd = torch.from_numpy(v).to("cuda")
    wd = torch.empty_like(vd)
    plan.pc_apply(vd, wd)
    torch.cuda.synchronize()
    err = float(np.abs(wd.cpu().numpy() - ref).max() / np.abs(ref).max())
    assert err < 1e-12, err
