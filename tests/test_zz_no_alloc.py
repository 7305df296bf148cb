"""wc_pc_apply_noalloc (no plan, no device allocation, tables and spectral workspace in a
static device array) against the plan-based wc_pc_apply on the same inputs: two calls in a
row, the second with a smaller problem, each to the parity bar of the preconditioner apply
(FP64 1e-12, FP32 2e-5 of max |w|)."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2406_00952_amd import wc
    return torch, wc


def relerr(a, b):
    return float((a - b).abs().max() / b.abs().max())


# pairs of calls: (dims, M, n, theta, method, precision) large first, then smaller
PAIRS = [
    ((2, 255, 256, 0.5, "gmres_ps", "fp64"), (2, 63, 64, 1.0, "gmres_ps", "fp64")),
    ((2, 127, 128, 0.5, "minres_abs_ps", "mixed"), (1, 63, 64, 0.5, "minres_abs_ps", "mixed")),
    ((1, 1023, 512, 1.0, "minres_pms", "fp64"), (2, 31, 16, 0.5, "minres_pms", "fp64")),
    ((2, 255, 128, 0.5, "gmres_ps", "mixed"), (2, 15, 8, 0.5, "gmres_ps", "mixed")),
]


@pytest.mark.parametrize("first,second", PAIRS)
def test_noalloc_matches_plan_apply(env, first, second):
    torch, wc = env
    for k, (dims, M, n, theta, method, precision) in enumerate((first, second)):
        print("noalloc", k, dims, M, n, theta, method, precision, flush=True)
        m = M ** dims
        v = torch.from_numpy(datagen.random_vector(21 + k, 2 * n * m)).cuda()
        ref = torch.empty_like(v)
        plan = wc.Plan(dims, M, n, theta=theta, gamma=1e-4, method=method, precision=precision)
        plan.pc_apply(v, ref)
        plan.close()
        w = torch.full_like(v, float("nan"))
        wc.pc_apply_noalloc(v, w, dims=dims, M=M, n=n, theta=theta, gamma=1e-4, method=method,
                            precision=precision)
        torch.cuda.synchronize()
        err = relerr(w, ref)
        print("  max rel diff", err, flush=True)
        assert err <= (1e-12 if precision == "fp64" else 2e-5)
        # in place, as wc_pc_apply allows
        wc.pc_apply_noalloc(v, v, dims=dims, M=M, n=n, theta=theta, gamma=1e-4, method=method,
                            precision=precision)
        torch.cuda.synchronize()
        assert relerr(v, ref) <= (1e-12 if precision == "fp64" else 2e-5)


def test_noalloc_rejects_beyond_limit(env):
    torch, wc = env
    assert wc.pc_apply_noalloc_limit() == 256 << 20
    v = torch.zeros(8, dtype=torch.float64, device="cuda")
    # 2D M = 511, n = 512 needs a 2.14 GB FP64 spectral array
    with pytest.raises(wc.WcError) as ei:
        wc.pc_apply_noalloc(v, v, dims=2, M=511, n=512, theta=0.5)
    assert ei.value.code == wc.WC_E_ARG
    with pytest.raises(wc.WcError) as ei:  # zeta != pi is not covered
        wc.pc_apply_noalloc(v, v, dims=2, M=63, n=64, theta=0.5, zeta=1.0)
    assert ei.value.code == wc.WC_E_UNSUPPORTED
