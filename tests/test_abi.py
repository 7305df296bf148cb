"""C-ABI checks that need no GPU: the library loads, exports every function
include/wc.h declares, and rejects invalid arguments before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2406_00952_amd", "lib", "libwcirc.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "wc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wc_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def wc():
    if not os.path.exists(LIB):
        pytest.fail("libwcirc.so is not built (run python -m paper_2406_00952_amd.build)")
    from paper_2406_00952_amd import wc as mod
    return mod


def test_library_exports_every_declared_symbol(wc):
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(wc.EXPORTED)


def test_status_strings(wc):
    assert wc.status_str(0) == "ok"
    assert "argument" in wc.status_str(1)
    assert wc.version().startswith("libwcirc")


@pytest.mark.parametrize("bad", [
    dict(dims=3), dict(M=0), dict(n=1), dict(theta=0.3), dict(theta=1.2), dict(gamma=0.0),
    dict(gamma=-1.0), dict(T=0.0), dict(tol=0.0), dict(restart=0), dict(restart=33),
    dict(maxit=0), dict(gamma=float("nan")),
])
def test_invalid_arguments_rejected(wc, bad):
    args = dict(dims=2, M=31, n=32, T=1.0, theta=0.5, gamma=1e-4)
    args.update(bad)
    assert wc.footprint_bytes(**args) == 0


def test_abs_ps_requires_constant_coefficient(wc):
    a = np.ones(2 * 7 * 8)
    assert wc.footprint_bytes(2, 7, 8, a_face=a, method="minres_abs_ps") == 0
    assert wc.footprint_bytes(2, 7, 8, a_face=a, method="minres_pms") > 0
    assert wc.footprint_bytes(2, 7, 8, a_face=-a, method="minres_pms") == 0


def test_footprint_grows_with_restart_and_precision(wc):
    f30 = wc.footprint_bytes(2, 255, 256, restart=30)
    f10 = wc.footprint_bytes(2, 255, 256, restart=10)
    nvec = 2 * 256 * 255 * 255 * 8
    assert f30 - f10 == 20 * nvec
    fm = wc.footprint_bytes(2, 255, 256, restart=30, precision="mixed")
    # mixed: FP32 spectral arrays but a flexible basis (30 more vectors)
    assert fm > f30
    # MINRES: ten system vectors
    fmin = wc.footprint_bytes(2, 255, 256, method="minres_abs_ps")
    assert 10 * nvec < fmin < 10 * nvec + 2 * 256 * 255 * 255 * 16 * 2 + (64 << 20)


def test_fem_options_and_footprint(wc):
    """Finite elements (wc_disc): a == 1, no low-rank form; the plan holds one more FP64
    complex array of n*m for the sine transforms of the data and the solution, and no
    transposed copy of the spectral array (the preconditioner has no sine passes)."""
    fd = wc.footprint_bytes(2, 63, 64)
    fe = wc.footprint_bytes(2, 63, 64, disc="fem")
    assert fe - fd == 64 * 63 * 63 * 16
    fd = wc.footprint_bytes(2, 255, 256)
    fe = wc.footprint_bytes(2, 255, 256, disc="fem")
    # (finite differences at N1 >= 128 hold the transposed copy, n*M*N1 complex)
    assert fe - fd == 256 * 255 * 255 * 16 - 256 * 255 * 256 * 16
    a = np.ones(2 * 7 * 8)
    assert wc.footprint_bytes(2, 7, 8, a_face=a, method="minres_pms", disc="fem") == 0
    assert wc.footprint_bytes(2, 7, 8, lowrank=True, disc="fem") == 0
    assert wc.footprint_bytes(2, 7, 8, disc=2) == 0
    assert wc.footprint_bytes(1, 7, 8, method="minres_abs_ps", disc="fem") > 0


def test_neumann_kappa_options_and_footprint(wc):
    """Neumann data (wc_bc): GMRES-P_S, finite differences, constant a; the plan holds a
    second spectral array and C, C^{-1} in FP64 and FP32.  kappa: 0 reads as 1, negative or
    non-finite refused, only 0 or 1 beside a variable coefficient."""
    fd = wc.footprint_bytes(2, 31, 32)
    fn = wc.footprint_bytes(2, 31, 32, bc="neumann", kappa=1e-3)
    assert fn - fd == 32 * 31 * 31 * 16 + 2 * 31 * 31 * 12
    # Dirichlet data with M + 1 = 33 takes the general path: both spectral arrays hold all
    # n frequencies (twice the FFT path's), plus Phi and its inverse and the full
    # eigenvalue table in FP64 and FP32; the dense sine matrices match the cosine ones
    fg = wc.footprint_bytes(2, 32, 32)
    fn = wc.footprint_bytes(2, 32, 32, bc="neumann")
    assert fg - fn == 2 * 32 * 32 * 32 * 16 + (2 * 32 * 32 + 32) * 24
    for kw in (dict(method="minres_abs_ps"), dict(method="minres_pms"), dict(lowrank=True),
               dict(disc="fem")):
        assert wc.footprint_bytes(2, 32, 32, bc="neumann", **kw) == 0, kw
    assert wc.footprint_bytes(2, 1, 32, bc="neumann") == 0      # M >= 2 nodes
    assert wc.footprint_bytes(2, 30, 32, bc="neumann") > 0      # any M
    assert wc.footprint_bytes(2, 31, 32, bc=2) == 0
    assert wc.footprint_bytes(2, 31, 32, kappa=0.0) == wc.footprint_bytes(2, 31, 32)
    assert wc.footprint_bytes(2, 31, 32, kappa=-1.0) == 0
    assert wc.footprint_bytes(2, 31, 32, kappa=float("nan")) == 0
    a = np.ones(2 * 31 * 32)
    assert wc.footprint_bytes(2, 31, 32, a_face=a, kappa=2.0) == 0
    assert wc.footprint_bytes(2, 31, 32, a_face=a, kappa=1.0) > 0


def test_multigrid_options_and_footprint(wc):
    a = np.ones(2 * 31 * 32)
    base = wc.footprint_bytes(2, 31, 32, method="gmres_ps")
    fa = wc.footprint_bytes(2, 31, 32, a_face=a, method="gmres_ps")
    spec = 32 * 31 * 31 * 16
    # the fine multigrid solution, coarse levels (about a third of it) and the face pyramid
    assert base + spec < fa < base + 2 * spec
    assert wc.footprint_bytes(2, 31, 32, a_face=a, mg_max_cycles=0) == 0
    assert wc.footprint_bytes(2, 31, 32, a_face=a, mg_tol=-1.0) == 0
    assert wc.footprint_bytes(2, 31, 32, a_face=a, mg_tol=0.0) > 0


def test_server_null_arguments(wc):
    lib = ctypes.CDLL(LIB)
    lib.wc_server_destroy.argtypes = [ctypes.c_void_p]
    lib.wc_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    lib.wc_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    lib.wc_server_bytes_in_use.argtypes = [ctypes.c_void_p]
    lib.wc_server_bytes_in_use.restype = ctypes.c_size_t
    lib.wc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    assert lib.wc_server_destroy(None) == wc.WC_E_ARG
    done = ctypes.c_int(0)
    assert lib.wc_server_poll(None, 1, ctypes.byref(done), None) == wc.WC_E_ARG
    assert lib.wc_server_cancel(None, 1) == wc.WC_E_ARG
    assert lib.wc_server_bytes_in_use(None) == 0
    h = ctypes.c_void_p()
    assert lib.wc_server_create(0, 0, ctypes.byref(h)) == wc.WC_E_ARG  # no workers
    assert lib.wc_server_create(0, 65, ctypes.byref(h)) == wc.WC_E_ARG


def test_retarget_null_plan(wc):
    lib = ctypes.CDLL(LIB)
    lib.wc_plan_retarget.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.wc_plan_retarget(None, None, None) == wc.WC_E_ARG


def test_lowrank_options_and_footprint(wc):
    full = wc.footprint_bytes(2, 255, 256, method="gmres_ps", restart=30)
    lr = wc.footprint_bytes(2, 255, 256, method="gmres_ps", restart=30, lowrank=True)
    nvec = 2 * 256 * 255 * 255 * 8
    assert 0 < lr < full - 25 * nvec  # the basis is compact: ~4 system vectors instead of ~35
    assert wc.footprint_bytes(2, 31, 32, method="minres_abs_ps", lowrank=True) == 0
    assert wc.footprint_bytes(1, 31, 32, method="gmres_ps", precision="mixed", lowrank=True) == 0
    mixed = wc.footprint_bytes(2, 255, 256, method="gmres_ps", precision="mixed", lowrank=True)
    assert 0 < mixed < lr  # 2D: the same compact basis with an FP32 spectral array
    a = np.ones(2 * 31 * 32)
    assert wc.footprint_bytes(2, 31, 32, method="gmres_ps", a_face=a, lowrank=True) == 0


def test_batch_null_arguments(wc):
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.wc_batch_create.argtypes = [vp, ctypes.c_int, vp]
    lib.wc_batch_destroy.argtypes = [vp]
    lib.wc_batch_pc_apply.argtypes = [vp, vp, vp]
    lib.wc_batch_solve.argtypes = [vp] * 7
    h = vp()
    assert lib.wc_batch_create(None, 1, ctypes.byref(h)) == wc.WC_E_ARG
    plans = (vp * 2)(None, None)
    assert lib.wc_batch_create(plans, 0, ctypes.byref(h)) == wc.WC_E_ARG   # empty batch
    assert lib.wc_batch_create(plans, 33, ctypes.byref(h)) == wc.WC_E_ARG  # above 32
    assert lib.wc_batch_create(plans, 2, ctypes.byref(h)) == wc.WC_E_ARG   # null plans
    assert lib.wc_batch_create(plans, 1, None) == wc.WC_E_ARG
    assert lib.wc_batch_destroy(None) == wc.WC_E_ARG
    assert lib.wc_batch_pc_apply(None, None, None) == wc.WC_E_ARG
    assert lib.wc_batch_solve(None, None, None, None, None, None, None) == wc.WC_E_ARG


def _create_plan_host(wc, **kw):
    """wc_plan_create through ctypes with no stream (only host-side refusals are checked)."""
    args = dict(dims=1, M=7, n=7, T=1.0, theta=0.5, gamma=1e-4, zeta=np.pi, s2_remedy=0.0,
                a_face=None)
    args.update(kw)
    pr, _keep = wc._problem(args["dims"], args["M"], args["n"], args["T"], args["theta"],
                            args["gamma"], args["zeta"], args["s2_remedy"], args["a_face"])
    op = wc._opts("gmres_ps", "fp64", 1e-8, 500, 30, False, 30, 1e-10)
    h = ctypes.c_void_p(1)
    code = wc._lib.wc_plan_create(ctypes.byref(pr), ctypes.byref(op), None, ctypes.byref(h))
    return code, h.value


@pytest.mark.parametrize("n,zeta", [(7, np.pi), (5, np.pi), (8, 0.0), (6, 0.0)])
def test_singular_s2_without_remedy_refused(wc, n, zeta):
    # remark on the singular S_n^(2) (Section 1): theta = 1/2 makes S^(2) singular when
    # e^{i(zeta - 2 pi l)/n} = -1 for some l: n odd at zeta = pi, n even at zeta = 0.
    # With s2_remedy = 0 plan creation fails before any device call and sets *out = NULL.
    code, h = _create_plan_host(wc, n=n, zeta=zeta)
    assert code == wc.WC_E_SINGULAR_S2 and h is None
    # the same problem with a remedy value is a valid problem
    assert wc.footprint_bytes(1, 7, n, theta=0.5, zeta=zeta, s2_remedy=1.0) > 0


def test_footprint_partials_cover_restart_32(wc):
    # GMRES step j < restart writes (j + 2) rows of 1024 reduction partials; with restart 32
    # that is 34 rows.  On a tiny problem the partials dominate the non-table bytes, so the
    # footprint is checked term by term (spectral array, partials, 1 MiB of tables,
    # (restart+1) + 1 + 1 + 2 system vectors, 512 Krylov scalars).
    M, n, k = 3, 4, 32
    nvec = 2 * n * M
    expect = n * M * 16 + (34 * 1024 + 64) * 8 + (1 << 20) + (k + 1 + 1 + 1 + 2) * nvec * 8 + 512 * 8
    assert wc.footprint_bytes(1, M, n, restart=k) == expect
