"""GPU tests of the solve server (include/wc.h, serving): a request's result is the same
whether it runs alone or in a concurrent mix (bitwise: every reduction has a fixed
order), admission keeps the held plans within the memory budget, and queued requests
can be cancelled."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

# dims, M, n, theta, gamma, method, precision, coeff
MIX = [
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const"),
    (2, 31, 32, 1.0, 1e-2, "minres_abs_ps", "fp64", "const"),
    (1, 255, 128, 0.5, 1e-6, "gmres_ps", "mixed", "const"),
    (2, 31, 64, 0.5, 1e-4, "gmres_ps", "fp64", "sin"),
    (2, 127, 64, 1.0, 1e-3, "gmres_ps", "mixed", "const"),
    (1, 127, 64, 1.0, 1e-4, "minres_pms", "fp64", "sin"),
    (2, 63, 32, 0.5, 1e-5, "minres_pms", "mixed", "const"),
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const"),  # same as the first: plan reuse
]


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_00952_amd import wc
    return torch, wc


def make_request(torch, k, spec):
    dims, M, n, theta, gamma, method, precision, coeff = spec
    d = datagen.config_problem(dims, M, n, seed=100 + k, noise_sigma=1e-3)
    a_face = datagen.sinusoidal_a(dims, M) if coeff == "sin" else None
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    m = M ** dims
    kw = dict(dims=dims, M=M, n=n, theta=theta, gamma=gamma, method=method,
              precision=precision, a_face=a_face)
    return kw, dev(d["f"]), dev(d["g"]), dev(d["y0"]), m


# low-rank GMRES requests (a = 1; FP32 preconditioner in 2D only)
MIX_LR = [
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const"),
    (2, 127, 64, 1.0, 1e-3, "gmres_ps", "mixed", "const"),
    (1, 255, 128, 0.5, 1e-6, "gmres_ps", "fp64", "const"),
    (2, 31, 32, 1.0, 1e-2, "gmres_ps", "fp64", "const"),
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const"),  # same as the first: plan reuse
]


def test_alone_equals_in_mix(env):
    _alone_equals_in_mix(env, MIX, False)


def test_alone_equals_in_mix_lowrank(env):
    _alone_equals_in_mix(env, MIX_LR, True)


def _alone_equals_in_mix(env, mix, lowrank):
    torch, wc = env
    reqs = [make_request(torch, k, s) for k, s in enumerate(mix)]
    for r in reqs:
        r[0]["lowrank"] = lowrank
    alone = []
    for kw, f, g, y0, m in reqs:
        y = torch.empty(kw["n"] * m, dtype=torch.float64, device="cuda")
        p = torch.empty_like(y)
        plan = wc.Plan(**kw)
        info = plan.solve(f, g, y0, y, p)
        assert info.relres <= 1e-8
        alone.append((y.cpu().numpy(), p.cpu().numpy(), info.iters))
        plan.close()
    torch.cuda.synchronize()
    srv = wc.Server(hbm_budget=0, max_concurrency=4)
    outs, tickets = [], []
    for kw, f, g, y0, m in reqs:
        y = torch.full((kw["n"] * m,), float("nan"), dtype=torch.float64, device="cuda")
        p = torch.full_like(y, float("nan"))
        outs.append((y, p))
    torch.cuda.synchronize()
    for (kw, f, g, y0, m), (y, p) in zip(reqs, outs):
        tickets.append(srv.submit(f, g, y0, y, p, **kw))
    for k, t in enumerate(tickets):
        info, q_ms, tot_ms = srv.wait(t)
        print("request", k, mix[k], "lowrank", lowrank, "iters", info.iters, "queue ms",
              round(q_ms, 2),
              "total ms", round(tot_ms, 2), flush=True)
        assert info.status == wc.WC_OK
        assert info.iters == alone[k][2]
        assert tot_ms >= q_ms >= 0.0
    torch.cuda.synchronize()
    for k, (y, p) in enumerate(outs):
        assert np.array_equal(y.cpu().numpy(), alone[k][0]), k
        assert np.array_equal(p.cpu().numpy(), alone[k][1]), k
    srv.close()


def test_admission_budget_and_cancel(env):
    torch, wc = env
    spec = (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const")
    kw, f, g, y0, m = make_request(torch, 0, spec)
    fp = wc.footprint_bytes(kw["dims"], kw["M"], kw["n"], theta=kw["theta"], gamma=kw["gamma"])
    # room for one plan only: requests run one after another, the plan is reused
    srv = wc.Server(hbm_budget=int(fp * 1.5), max_concurrency=4)
    outs = [(torch.empty(kw["n"] * m, dtype=torch.float64, device="cuda"),
             torch.empty(kw["n"] * m, dtype=torch.float64, device="cuda")) for _ in range(4)]
    tickets = [srv.submit(f, g, y0, y, p, **kw) for (y, p) in outs]
    cancelled = srv.cancel(tickets[-1])
    results = [srv.wait(t) for t in tickets]
    assert all(r[0].status == wc.WC_OK for r in results[:3])
    if cancelled:
        assert results[3][0].status == wc.WC_E_CANCELLED
    assert srv.bytes_in_use() <= int(fp * 1.5)
    # a request larger than the budget is refused at submission
    big = dict(kw, M=127, n=128)
    fb = torch.empty(129 * 127 * 127, dtype=torch.float64, device="cuda")
    yb = torch.empty(128 * 127 * 127, dtype=torch.float64, device="cuda")
    with pytest.raises(wc.WcError) as ei:
        srv.submit(fb, fb, fb[: 127 * 127].contiguous(), yb, yb.clone(), **big)
    assert ei.value.code == wc.WC_E_ADMISSION
    srv.close()


@pytest.mark.parametrize("coeff", ["const", "sin"])
def test_retarget_matches_fresh_plan(env, coeff):
    """A plan retargeted to another problem of the same shape gives bitwise the result of
    a plan created for that problem."""
    torch, wc = env
    dims, M, n = 2, 31, 32
    kw, f, g, y0, m = make_request(torch, 5, (dims, M, n, 0.5, 1e-4, "gmres_ps", "fp64", coeff))
    a2 = None
    if coeff == "sin":
        a2 = 1.0 + 0.25 * (datagen.sinusoidal_a(dims, M) - 1.0)
    target = dict(T=2.0, theta=1.0, gamma=3e-3, a_face=a2)
    y1 = torch.empty(n * m, dtype=torch.float64, device="cuda")
    p1, y2, p2 = torch.empty_like(y1), torch.empty_like(y1), torch.empty_like(y1)
    fresh = wc.Plan(dims, M, n, method="gmres_ps", **target)
    i1 = fresh.solve(f, g, y0, y1, p1)
    plan = wc.Plan(**kw)
    plan.solve(f, g, y0, y2, p2)
    plan.retarget(**target)
    i2 = plan.solve(f, g, y0, y2, p2)
    torch.cuda.synchronize()
    assert i1.iters == i2.iters and i1.relres == i2.relres
    assert np.array_equal(y1.cpu().numpy(), y2.cpu().numpy())
    assert np.array_equal(p1.cpu().numpy(), p2.cpu().numpy())
    with pytest.raises(wc.WcError):
        plan.retarget(theta=0.5, gamma=1e-4, a_face=None if coeff == "sin" else
                      datagen.sinusoidal_a(dims, M))
