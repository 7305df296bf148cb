"""GPU tests of the solve server (include/wc.h, serving): a request's result is the same
whether it is served alone or in a concurrent mix (bitwise: every reduction has a fixed
order and the batched kernels' work units read one instance each), it matches the
standalone solve of the same problem, requests of the batchable kind really are
continuously batched (several active in one round, joining while others run), admission
keeps the held plans within the memory budget, and queued requests can be cancelled."""
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


def _serve(wc, torch, reqs, lowrank, idx=None):
    """Submits reqs (all, or those listed in idx) to a fresh server at once; returns
    [(y, p, info)] in order and the server's batching statistics."""
    idx = range(len(reqs)) if idx is None else idx
    srv = wc.Server(hbm_budget=0, max_concurrency=4)
    outs, tickets = [], []
    for k in idx:
        kw, f, g, y0, m = reqs[k]
        y = torch.full((kw["n"] * m,), float("nan"), dtype=torch.float64, device="cuda")
        outs.append((y, torch.full_like(y, float("nan"))))
    torch.cuda.synchronize()
    for k, (y, p) in zip(idx, outs):
        kw, f, g, y0, m = reqs[k]
        tickets.append(srv.submit(f, g, y0, y, p, **dict(kw, lowrank=lowrank)))
    res = []
    for t, (y, p) in zip(tickets, outs):
        info, q_ms, tot_ms = srv.wait(t)
        assert tot_ms >= q_ms >= 0.0
        res.append((y.cpu().numpy(), p.cpu().numpy(), info))
    stats = srv.stats()
    srv.close()
    return res, stats


def _alone_equals_in_mix(env, mix, lowrank):
    torch, wc = env
    reqs = [make_request(torch, k, s) for k, s in enumerate(mix)]
    mixed, stats = _serve(wc, torch, reqs, lowrank)
    print("batched requests, most active in one round:", stats, flush=True)
    for k, (kw, f, g, y0, m) in enumerate(reqs):
        alone, _ = _serve(wc, torch, reqs, lowrank, [k])
        ya, pa, ia = alone[0]
        ym, pm, im = mixed[k]
        print("request", k, mix[k], "lowrank", lowrank, "iters", im.iters, flush=True)
        assert im.status == wc.WC_OK and ia.status == wc.WC_OK and im.relres <= 1e-8
        assert im.iters == ia.iters
        assert np.array_equal(ym, ya), k
        assert np.array_equal(pm, pa), k
        # the same problem through a standalone plan (single-instance kernels)
        y = torch.empty(kw["n"] * m, dtype=torch.float64, device="cuda")
        p = torch.empty_like(y)
        plan = wc.Plan(**dict(kw, lowrank=lowrank))
        info = plan.solve(f, g, y0, y, p)
        plan.close()
        assert info.iters == im.iters
        sc = max(np.abs(ym).max(), np.abs(pm).max())
        assert np.abs(y.cpu().numpy() - ym).max() <= 1e-10 * sc
        assert np.abs(p.cpu().numpy() - pm).max() <= 1e-10 * sc


# requests the server batches continuously (2D, a = 1, standard GMRES(k)-P_S, n and M+1 in
# {64, ..., 512}), mixed sizes and precisions
MIX_CB = [
    (2, 63, 64, 0.5, 1e-4, "gmres_ps", "fp64", "const"),
    (2, 127, 128, 1.0, 1e-3, "gmres_ps", "mixed", "const"),
    (2, 63, 128, 0.5, 1e-6, "gmres_ps", "fp64", "const"),
    (2, 255, 64, 0.5, 1e-2, "gmres_ps", "fp64", "const"),
    (2, 127, 64, 1.0, 1e-5, "gmres_ps", "mixed", "const"),
    (2, 63, 64, 1.0, 1e-3, "gmres_ps", "fp64", "const"),
]


def test_continuous_batching(env):
    """Requests arrive while others iterate: they join the running lockstep rounds, several
    solves are active in one round, every batchable request is served by the batcher, and
    each result is bitwise the one served alone."""
    torch, wc = env
    reqs = [make_request(torch, 20 + k, s) for k, s in enumerate(MIX_CB)]
    alone = [_serve(wc, torch, reqs, False, [k])[0][0] for k in range(len(reqs))]
    srv = wc.Server(hbm_budget=0, max_concurrency=2)
    outs, tickets = [], []
    import time
    for k, (kw, f, g, y0, m) in enumerate(reqs):
        y = torch.full((kw["n"] * m,), float("nan"), dtype=torch.float64, device="cuda")
        p = torch.full_like(y, float("nan"))
        outs.append((y, p))
        torch.cuda.synchronize()
        tickets.append(srv.submit(f, g, y0, y, p, **kw))
        time.sleep(0.002)  # staggered arrivals: later requests join running rounds
    for k, t in enumerate(tickets):
        info, q_ms, tot_ms = srv.wait(t)
        y, p = outs[k]
        assert info.status == wc.WC_OK and info.relres <= 1e-8
        assert info.iters == alone[k][2].iters
        assert np.array_equal(y.cpu().numpy(), alone[k][0]), k
        assert np.array_equal(p.cpu().numpy(), alone[k][1]), k
    batched, most = srv.stats()
    print("batched", batched, "most active in one round", most, flush=True)
    assert batched == len(reqs)
    assert most >= 2
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


def test_plan_reuse_across_zeta(env):
    """Requests of one shape at zeta = pi and zeta = 1 take different preconditioner paths
    (the half-spectrum FFT path and the general path), so the idle plan of the first is not
    retargeted to the second: both succeed, and the second equals its standalone solve."""
    torch, wc = env
    dims, M, n = 2, 31, 32
    kw, f, g, y0, m = make_request(torch, 7, (dims, M, n, 0.5, 1e-4, "gmres_ps", "fp64", "const"))
    print("server zeta pi then zeta 1", dims, M, n, flush=True)
    srv = wc.Server(hbm_budget=0, max_concurrency=1)
    outs = [(torch.empty(n * m, dtype=torch.float64, device="cuda"),
             torch.empty(n * m, dtype=torch.float64, device="cuda")) for _ in range(2)]
    r0 = srv.wait(srv.submit(f, g, y0, *outs[0], **kw))
    r1 = srv.wait(srv.submit(f, g, y0, *outs[1], **dict(kw, zeta=1.0)))
    srv.close()
    assert r0[0].status == wc.WC_OK and r1[0].status == wc.WC_OK
    assert r1[0].relres <= 1e-8
    plan = wc.Plan(**dict(kw, zeta=1.0))
    y = torch.empty(n * m, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    info = plan.solve(f, g, y0, y, p)
    torch.cuda.synchronize()
    assert info.iters == r1[0].iters
    assert np.array_equal(y.cpu().numpy(), outs[1][0].cpu().numpy())
    assert np.array_equal(p.cpu().numpy(), outs[1][1].cpu().numpy())
