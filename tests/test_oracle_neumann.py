"""Pins of the oracle's Neumann form (Example 3 of Section 4: homogeneous Neumann data,
constant a) and of the constant-coefficient scale kappa, CPU only.

* K is the ghost-node definition, written here entry by entry from the mirrored
  neighbours, and annihilates constants (pure Neumann data);
* the cosine matrix C holds eigenvectors of K with the closed-form eigenvalues, and the
  weighted-transpose inverse equals the numerical inverse;
* the three-step P_S apply equals the dense inverse of P_S built from its definition
  (K in both block rows);
* GMRES-P_S equals the sparse direct solve of A_tilde;
* Table 4 (h = 2^-5 and 2^-6, all five gamma): 3 iterations and e_h to the printed
  three digits (fixture tests/golden/table4_example3_cn.txt);
* the discrete solution converges at second order (ratio about 4 per halving);
* kappa scales K (and the sine-path apply) for Dirichlet data.
"""
import numpy as np
import pytest

import datagen
from oracle import spatial, solver
from oracle.discretization import Problem, AllAtOnce, stiffness_neumann, mass_stiffness
from oracle.precond import FastPreconditioner, dense_PS
from conftest import load_golden


def _ghost_K1(M, kappa):
    """(K1 u)_j = kappa (2 u_j - u_{j-1} - u_{j+1}) / h^2 with u_{-1} = u_1, u_M = u_{M-2}."""
    h = 1.0 / (M - 1)
    K = np.zeros((M, M))
    for j in range(M):
        for nb in (j - 1, j + 1):
            nb = 1 if nb == -1 else (M - 2 if nb == M else nb)  # mirrored ghost nodes
            K[j, nb] -= kappa / h ** 2
        K[j, j] += 2 * kappa / h ** 2
    return K


@pytest.mark.parametrize("M", [2, 3, 8])
def test_neumann_K_is_ghost_node_definition(M):
    K1 = _ghost_K1(M, 0.3)
    np.testing.assert_allclose(stiffness_neumann(1, M, 0.3).toarray(), K1, rtol=1e-14)
    K2 = np.kron(np.eye(M), K1) + np.kron(K1, np.eye(M))  # x2 index outer
    np.testing.assert_allclose(stiffness_neumann(2, M, 0.3).toarray(), K2, rtol=1e-14)
    # constants are in the null space; K is not symmetric for M > 2
    np.testing.assert_allclose(stiffness_neumann(2, M, 0.3) @ np.ones(M * M), 0.0, atol=1e-9)
    if M > 2:
        assert np.abs(K1 - K1.T).max() > 0


@pytest.mark.parametrize("M", [3, 5, 9])
def test_cosine_basis_diagonalises(M):
    C = spatial.cosine_matrix(M)
    Ci = spatial.cosine_inverse(M)
    np.testing.assert_allclose(Ci, np.linalg.inv(C), atol=1e-12)
    for dims in (1, 2):
        K = stiffness_neumann(dims, M, 1.0).toarray()
        V = C if dims == 1 else np.kron(C, C)
        lam = spatial.neumann_eigenvalues(dims, M)
        np.testing.assert_allclose(K @ V, V * lam[None, :], atol=1e-9 * np.abs(K).max())
        X = np.random.default_rng(0).standard_normal((2, M ** dims))
        Y = spatial.cosine_transform(dims, M, X, inverse=True)
        np.testing.assert_allclose(Y, X @ np.linalg.inv(V).T, atol=1e-11)
        np.testing.assert_allclose(spatial.cosine_transform(dims, M, Y, inverse=False), X,
                                   atol=1e-11)


@pytest.mark.parametrize("dims,M,n,theta", [(1, 6, 4, 0.5), (2, 4, 4, 1.0), (2, 3, 6, 0.5)])
def test_neumann_fast_ps_matches_dense(dims, M, n, theta):
    pr = Problem(dims=dims, M=M, n=n, theta=theta, gamma=1e-2, bc="neumann", kappa=0.7)
    P = dense_PS(pr)
    v = np.random.default_rng(3).standard_normal(2 * n * pr.m)
    ref = np.linalg.solve(P, v).real
    np.testing.assert_allclose(FastPreconditioner(pr, "ps").apply(v), ref,
                               atol=1e-11 * np.abs(ref).max())
    for kind in ("abs_ps", "pms"):
        with pytest.raises(ValueError):
            FastPreconditioner(pr, kind)


def test_neumann_system_not_symmetric():
    pr = Problem(dims=1, M=5, n=4, theta=0.5, gamma=1e-2, bc="neumann")
    op = AllAtOnce(pr)
    N = 2 * pr.n * pr.m
    A = np.column_stack([op.A(e) for e in np.eye(N)])
    assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()


@pytest.mark.parametrize("dims,M,n", [(1, 17, 16), (2, 9, 8)])
def test_neumann_gmres_matches_direct(dims, M, n):
    d = datagen.config_problem(dims, M, n, seed=8, noise_sigma=1e-3, y0_zero=False)
    pr = Problem(dims=dims, M=M, n=n, theta=0.5, gamma=1e-4, bc="neumann", kappa=0.1)
    y, p = solver.direct_solve(pr, d["f"], d["g"], d["y0"])
    out = solver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-12, maxit=300)
    sc = max(np.abs(y).max(), np.abs(p).max())
    np.testing.assert_allclose(out["y"], y, atol=1e-9 * sc)
    np.testing.assert_allclose(out["p"], p, atol=1e-9 * sc)


@pytest.mark.parametrize("hexp", [5, 6])
@pytest.mark.parametrize("gamma", [1e-10, 1e-8, 1e-6, 1e-4, 1e-2])
def test_table4_rows(hexp, gamma):
    row = [r for r in load_golden("table4_example3_cn.txt")
           if int(r[1]) == hexp and float(r[0]) == gamma][0]
    N = 2 ** hexp                         # nodes per dimension, n = N time steps
    d = datagen.example3(N, N)
    pr = Problem(dims=2, M=N, n=N, theta=0.5, gamma=gamma, bc="neumann", kappa=1e-3)
    assert 2 * pr.n * pr.m == int(row[2])
    out = solver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-8)
    eh = solver.e_h(pr, out["y"], out["p"], d["y_exact"], d["p_exact"])
    assert out["iters"] == int(row[3])
    assert float(f"{eh:.3g}") == pytest.approx(float(row[4]), rel=1e-9)


def test_neumann_second_order():
    errs = []
    for N in (9, 17, 33):
        d = datagen.example3(N, N - 1, kappa=0.05)
        pr = Problem(dims=2, M=N, n=N - 1, theta=0.5, gamma=1e-2, bc="neumann", kappa=0.05)
        out = solver.solve(pr, d["f"], d["g"], d["y0"], "gmres_ps", tol=1e-12, maxit=300)
        errs.append(solver.e_h(pr, out["y"], out["p"], d["y_exact"], d["p_exact"]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.6 < r2 < 4.4, errs


@pytest.mark.parametrize("disc", ["fd", "fem"])
def test_kappa_scales_stiffness_and_apply(disc):
    pr1 = Problem(dims=2, M=5, n=4, theta=0.5, gamma=1e-2, disc=disc)
    prk = Problem(dims=2, M=5, n=4, theta=0.5, gamma=1e-2, disc=disc, kappa=2.5)
    np.testing.assert_allclose(mass_stiffness(prk)[1].toarray(),
                               2.5 * mass_stiffness(pr1)[1].toarray(), rtol=1e-14)
    v = np.random.default_rng(5).standard_normal(2 * 4 * 25)
    ref = np.linalg.solve(dense_PS(prk), v).real
    np.testing.assert_allclose(FastPreconditioner(prk, "ps").apply(v), ref,
                               atol=1e-11 * np.abs(ref).max())


def test_problem_validation():
    with pytest.raises(ValueError):
        Problem(dims=2, M=8, n=4, bc="robin")
    with pytest.raises(ValueError):
        Problem(dims=2, M=8, n=4, bc="neumann", disc="fem")
    with pytest.raises(ValueError):
        Problem(dims=1, M=8, n=4, bc="neumann", a_face=np.ones(9))
    with pytest.raises(ValueError):
        Problem(dims=1, M=8, n=4, kappa=0.0)
    assert Problem(dims=1, M=33, n=4, bc="neumann").h == pytest.approx(1 / 32)
