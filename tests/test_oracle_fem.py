"""Pins of the oracle's finite element form (Section 1: M_m SPD mass, K_m stiffness, and
the change of variables of eqn:main_system with M_m^{-1/2} K_m M_m^{-1/2}), CPU only.

* the mass and stiffness matrices equal the element integrals of the hat functions,
  computed here by quadrature of the piecewise-linear basis;
* M^{+-1/2} through the sine basis equals the dense symmetric square root;
* the spectrum of M^{-1/2} K M^{-1/2} equals the closed form k_j/m_j (sums in 2D);
* A from the change of variables equals the block formula of eqn:matrix_A;
* the fast three-step applies equal the dense inverses of P_S, |P_S|, P_MS;
* every Krylov solve equals the sparse direct solve of A_tilde;
* the discrete solution converges at second order for the manufactured solution of
  Example 1 (exact y = e^{-t} sin(pi x1) sin(pi x2), p = 0).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import datagen
from oracle import circulant, spatial, solver
from oracle.discretization import (Problem, AllAtOnce, fem_matrices, mass_power, B1, B2,
                                   Bn_closed_form)
from oracle.precond import (FastPreconditioner, dense_PS, dense_absPS, dense_PMS, dense_khat)


def _hat_integrals(M, q=64):
    """Mass and stiffness of the 1D hat functions on (0, 1), h = 1/(M+1), by Gauss
    quadrature with q points per element (exact for the piecewise polynomials)."""
    h = 1.0 / (M + 1)
    xg, wg = np.polynomial.legendre.leggauss(q)
    mass = np.zeros((M, M))
    stiff = np.zeros((M, M))
    for e in range(M + 1):  # element [e h, (e+1) h]
        x = e * h + (xg + 1) * h / 2
        w = wg * h / 2
        phi, dphi = {}, {}
        for i in range(M):  # node (i+1) h
            xi = (i + 1) * h
            v = np.maximum(0.0, 1.0 - np.abs(x - xi) / h)
            if np.any(v > 0):
                phi[i] = v
                dphi[i] = np.where(np.abs(x - xi) < h, -np.sign(x - xi) / h, 0.0)
        for i in phi:
            for j in phi:
                mass[i, j] += np.sum(w * phi[i] * phi[j])
                stiff[i, j] += np.sum(w * dphi[i] * dphi[j])
    return mass, stiff


@pytest.mark.parametrize("M", [1, 3, 6])
def test_fem_matrices_are_element_integrals(M):
    m1, k1 = _hat_integrals(M)
    Mm, Km = fem_matrices(1, M)
    np.testing.assert_allclose(Mm.toarray(), m1, atol=1e-14)
    np.testing.assert_allclose(Km.toarray(), k1, rtol=1e-12, atol=1e-12)
    # bilinear: integrals of products of tensor hats factor into the 1D integrals
    M2, K2 = fem_matrices(2, M)
    np.testing.assert_allclose(M2.toarray(), np.kron(m1, m1), atol=1e-14)
    np.testing.assert_allclose(K2.toarray(), np.kron(k1, m1) + np.kron(m1, k1), rtol=1e-12,
                               atol=1e-12)


@pytest.mark.parametrize("dims,M", [(1, 7), (2, 5)])
@pytest.mark.parametrize("power", [0.5, -0.5])
def test_mass_power_is_dense_square_root(dims, M, power):
    pr = Problem(dims=dims, M=M, n=2, disc="fem")
    Mm, _ = fem_matrices(dims, M)
    w, V = np.linalg.eigh(Mm.toarray())
    ref = (V * w ** power) @ V.T
    X = np.random.default_rng(1).standard_normal((3, pr.m))
    np.testing.assert_allclose(mass_power(pr, X, power), X @ ref.T, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,M", [(1, 9), (2, 6)])
def test_khat_spectrum_closed_form(dims, M):
    pr = Problem(dims=dims, M=M, n=2, disc="fem")
    Kh = dense_khat(pr)
    np.testing.assert_allclose(Kh, Kh.T, atol=1e-10 * np.abs(Kh).max())
    ev = np.linalg.eigvalsh(0.5 * (Kh + Kh.T))
    np.testing.assert_allclose(np.sort(ev), np.sort(spatial.fem_eigenvalues(dims, M)),
                               rtol=1e-10)


@pytest.mark.parametrize("dims,M,n,theta", [(1, 5, 4, 0.5), (2, 3, 4, 1.0)])
def test_fem_operator_block_form(dims, M, n, theta):
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=3e-3, disc="fem")
    op = AllAtOnce(pr)
    N = 2 * n * pr.m
    E = np.eye(N)
    A = np.column_stack([op.A(E[:, j]) for j in range(N)])
    Kh = dense_khat(pr)
    Bn = Bn_closed_form(n, theta)
    Im, In = np.eye(pr.m), np.eye(n)
    T = np.kron(Bn, Im) + pr.tau * np.kron(In, Kh)
    a = pr.alpha
    ref = np.block([[a * np.eye(n * pr.m), T.T], [T, -a * np.eye(n * pr.m)]])
    np.testing.assert_allclose(A, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("dims,M,n,theta", [(1, 5, 4, 0.5), (2, 3, 4, 1.0), (2, 3, 6, 0.5)])
@pytest.mark.parametrize("kind,dense", [("ps", dense_PS), ("abs_ps", dense_absPS),
                                        ("pms", dense_PMS)])
def test_fem_fast_preconditioner_matches_dense(dims, M, n, theta, kind, dense):
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=1e-2, disc="fem")
    P = dense(pr)
    v = np.random.default_rng(7).standard_normal(2 * n * pr.m)
    ref = np.linalg.solve(P, v).real
    np.testing.assert_allclose(FastPreconditioner(pr, kind).apply(v), ref,
                               atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("dims,M,n,theta", [(1, 15, 16, 0.5), (2, 7, 8, 1.0), (2, 7, 8, 0.5)])
@pytest.mark.parametrize("method", ["gmres_ps", "minres_abs_ps", "minres_pms"])
def test_fem_krylov_matches_direct(dims, M, n, theta, method):
    d = datagen.config_problem(dims, M, n, seed=6, noise_sigma=1e-3, y0_zero=False)
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=1e-4, disc="fem")
    y, p = solver.direct_solve(pr, d["f"], d["g"], d["y0"])
    out = solver.solve(pr, d["f"], d["g"], d["y0"], method, tol=1e-12, maxit=400)
    sc = max(np.abs(y).max(), np.abs(p).max())
    np.testing.assert_allclose(out["y"], y, atol=1e-9 * sc)
    np.testing.assert_allclose(out["p"], p, atol=1e-9 * sc)


def test_fem_second_order_convergence():
    errs = []
    for e in (3, 4, 5):
        M, n = 2 ** e - 1, 2 ** e
        d = datagen.example1(M, n)
        pr = Problem(dims=2, M=M, n=n, theta=0.5, gamma=1e-2, disc="fem")
        y, p = solver.direct_solve(pr, d["f"], d["g"], d["y0"])
        errs.append(solver.e_h(pr, y, p, d["y_exact"], d["p_exact"]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    # the coarsest grid is not yet asymptotic; the last halving is close to 4
    assert r1 > 3.5 and 3.7 < r2 < 4.4, errs
