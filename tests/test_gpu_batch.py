"""GPU tests of batches (include/wc.h, batches): the preconditioner passes of several
instances of uneven (M, n), methods and precisions run as one launch per pass, and
GMRES(k)-P_S advanced in lockstep over a batch.  Each instance must give what the same
plan gives alone, to rounding (the tile bodies are the same code, compiled into other
kernels), with the same iteration counts, and the batched apply is also checked against
the oracle."""
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


MIX = [
    # M, n, theta, gamma, method, precision
    (63, 64, 0.5, 1e-4, "gmres_ps", "fp64"),
    (127, 128, 1.0, 1e-2, "minres_abs_ps", "fp64"),
    (255, 64, 0.5, 1e-6, "minres_pms", "mixed"),
    (63, 512, 0.5, 1e-4, "gmres_ps", "mixed"),
    (511, 64, 1.0, 1e-4, "gmres_ps", "fp64"),
    (127, 256, 0.5, 1e-3, "gmres_ps", "fp64"),
]


def _plans(wc, cases, **kw):
    return [wc.Plan(2, M, n, theta=th, gamma=ga, method=me, precision=pr, **kw)
            for (M, n, th, ga, me, pr) in cases]


def test_batch_pc_apply_matches_single(env):
    torch, wc = env
    print("batch pc_apply", len(MIX), "instances", flush=True)
    plans = _plans(wc, MIX)
    batch = wc.Batch(plans)
    vs, ws, refs = [], [], []
    for i, (M, n, *_r) in enumerate(MIX):
        v = torch.from_numpy(datagen.random_vector(20 + i, 2 * n * M * M)).to("cuda")
        w1 = torch.empty_like(v)
        plans[i].pc_apply(v, w1)
        vs.append(v)
        ws.append(torch.full_like(v, float("nan")))
        refs.append(w1)
    batch.pc_apply(vs, ws)
    torch.cuda.synchronize()
    for i, case in enumerate(MIX):
        a, b = ws[i].cpu().numpy(), refs[i].cpu().numpy()
        sc = np.abs(b).max()
        err = np.abs(a - b).max() / sc
        print("  ", case, "max rel diff to the single apply", err, flush=True)
        assert np.isfinite(a).all()
        # the single-instance path may take other kernels for the same arithmetic (the
        # transposed x2 pass, per-block-row time passes), so rounding orders differ
        assert err <= (1e-14 if case[5] == "fp64" else 1e-5), (case, err)
    batch.close()


def test_batch_pc_apply_matches_oracle(env):
    torch, wc = env
    cases = [(63, 64, 0.5, 1e-4, "gmres_ps", "fp64"), (127, 128, 1.0, 1e-2, "minres_abs_ps", "fp64"),
             (63, 128, 0.5, 1e-6, "minres_pms", "fp64")]
    plans = _plans(wc, cases)
    batch = wc.Batch(plans)
    vs, ws, vnp = [], [], []
    for i, (M, n, *_r) in enumerate(cases):
        v = datagen.random_vector(40 + i, 2 * n * M * M)
        vnp.append(v)
        vs.append(torch.from_numpy(v).to("cuda"))
        ws.append(torch.empty_like(vs[-1]))
    batch.pc_apply(vs, ws)
    torch.cuda.synchronize()
    for i, (M, n, th, ga, me, pr) in enumerate(cases):
        kind = {"gmres_ps": "ps", "minres_abs_ps": "abs_ps", "minres_pms": "pms"}[me]
        ref = FastPreconditioner(Problem(dims=2, M=M, n=n, theta=th, gamma=ga), kind).apply(vnp[i])
        err = float(np.abs(ws[i].cpu().numpy() - ref).max() / np.abs(ref).max())
        print("  oracle", cases[i], err, flush=True)
        assert err < 1e-12, err


SOLVE = [
    # M, n, theta, gamma, precision, restart, seed
    (63, 64, 0.5, 1e-4, "fp64", 30, 0),
    (127, 128, 1.0, 1e-2, "mixed", 30, 1),
    (63, 256, 0.5, 1e-6, "fp64", 4, 2),     # several restart cycles
    (255, 64, 0.5, 1e-4, "fp64", 30, 3),
]


def _data(torch, M, n, seed):
    d = datagen.config_problem(2, M, n, seed=seed, noise_sigma=1e-3)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return dev(d["f"]), dev(d["g"]), dev(d["y0"])


def test_batch_solve_matches_single(env):
    torch, wc = env
    print("batch solve", len(SOLVE), "instances", flush=True)
    plans = [wc.Plan(2, M, n, theta=th, gamma=ga, method="gmres_ps", precision=pr, restart=rs,
                     tol=1e-8, maxit=400) for (M, n, th, ga, pr, rs, _s) in SOLVE]
    data = [_data(torch, M, n, sd) for (M, n, _t, _g, _p, _r, sd) in SOLVE]
    single = []
    for pl, (f, g, y0), (M, n, *_r) in zip(plans, data, SOLVE):
        y = torch.empty(n * M * M, dtype=torch.float64, device="cuda")
        p = torch.empty_like(y)
        info = pl.solve(f, g, y0, y, p)
        single.append((info, y.cpu().numpy(), p.cpu().numpy()))
    batch = wc.Batch(plans)
    for rep in range(2):  # a second run reuses every workspace
        ys = [torch.full((n * M * M,), float("nan"), dtype=torch.float64, device="cuda")
              for (M, n, *_r) in SOLVE]
        ps = [torch.full_like(y, float("nan")) for y in ys]
        infos = batch.solve([d[0] for d in data], [d[1] for d in data], [d[2] for d in data],
                            ys, ps)
        for i, case in enumerate(SOLVE):
            si, sy, sp = single[i]
            bi = infos[i]
            print("  ", rep, case, "iters", bi.iters, "single", si.iters, "restarts", bi.restarts,
                  "relres", bi.relres, flush=True)
            assert bi.status == wc.WC_OK and bi.relres <= 1e-8
            assert bi.iters == si.iters and bi.restarts == si.restarts
            sc = max(np.abs(sy).max(), np.abs(sp).max())
            # FP64: the same arithmetic in another order; mixed: the batched and single FP32
            # applies round differently (1e-7 per apply), so the two solutions agree to about
            # the solve tolerance
            bound = (1e-11 if case[4] == "fp64" else 1e-8) * sc
            assert np.abs(ys[i].cpu().numpy() - sy).max() <= bound
            assert np.abs(ps[i].cpu().numpy() - sp).max() <= bound
    batch.close()


def test_batch_many_rhs(env):
    """Eight right-hand sides of one problem (eight plans of it) in one batch."""
    torch, wc = env
    M, n = 127, 64
    plans = [wc.Plan(2, M, n, theta=0.5, gamma=1e-4, method="gmres_ps", tol=1e-8) for _ in range(8)]
    data = [_data(torch, M, n, 100 + s) for s in range(8)]
    ys = [torch.empty(n * M * M, dtype=torch.float64, device="cuda") for _ in range(8)]
    ps = [torch.empty_like(y) for y in ys]
    batch = wc.Batch(plans)
    infos = batch.solve([d[0] for d in data], [d[1] for d in data], [d[2] for d in data], ys, ps)
    for s in range(8):
        ref_y = torch.empty_like(ys[s])
        ref_p = torch.empty_like(ys[s])
        ri = plans[s].solve(*data[s], ref_y, ref_p)
        assert infos[s].relres <= 1e-8 and infos[s].iters == ri.iters
        # the batched passes round differently from the single ones (at N1 >= 128 the single
        # plan's x2 pass works on the transposed copy): ulp-level differences per apply,
        # carried through the iterations as in test_batch_solve_matches_single
        sc = max(float(ref_y.abs().max()), float(ref_p.abs().max()))
        dy = float((ys[s] - ref_y).abs().max()) / sc
        dp = float((ps[s] - ref_p).abs().max()) / sc
        assert dy <= 1e-11 and dp <= 1e-11, (s, dy, dp)
    print("  many rhs iters", [i.iters for i in infos], "ms", infos[0].ms, flush=True)
    batch.close()


def test_batch_rejects_unsupported(env):
    torch, wc = env
    with pytest.raises(wc.WcError):
        wc.Batch([wc.Plan(1, 63, 64)])                      # 1D
    with pytest.raises(wc.WcError):
        wc.Batch([wc.Plan(2, 31, 64)])                      # M + 1 = 32 is outside the set
    with pytest.raises(wc.WcError):
        wc.Batch([wc.Plan(2, 63, 1024)])                    # n = 1024
    with pytest.raises(wc.WcError):
        a = datagen.sinusoidal_a(2, 63)
        wc.Batch([wc.Plan(2, 63, 64, a_face=a, method="gmres_ps")])  # variable a
    pl = wc.Plan(2, 63, 64)
    with pytest.raises(wc.WcError):
        wc.Batch([pl, pl])                                  # one workspace per instance
    mr = wc.Plan(2, 63, 64, method="minres_abs_ps")
    b = wc.Batch([mr])
    f, g, y0 = _data(torch, 63, 64, 0)
    y = torch.empty(64 * 63 * 63, dtype=torch.float64, device="cuda")
    p = torch.empty_like(y)
    with pytest.raises(wc.WcError):
        b.solve([f], [g], [y0], [y], [p])                   # lockstep solve is GMRES only
    b.close()
