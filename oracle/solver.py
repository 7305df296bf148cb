"""End-to-end oracle solve of the discrete optimality system.

Methods (Section 4 naming):
  "minres_abs_ps" -- MINRES on A (eqn:main_system) with |P_S|
  "minres_pms"    -- MINRES on A with P_MS
  "gmres_ps"      -- GMRES on A_hat (eqn:main_system_nonsym) with P_S
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla
import scipy.linalg as sla

from .discretization import (Problem, AllAtOnce, rhs_tilde, transformed_rhs,
                             assemble_Atilde, B2, mass_power)
from .precond import FastPreconditioner
from . import krylov

METHODS = {"minres_abs_ps": ("abs_ps", True), "minres_pms": ("pms", True),
           "gmres_ps": ("ps", False)}


def recover(prob: Problem, x: np.ndarray):
    """x = [sqrt(gamma) y_tilde; p_tilde] -> y (levels 1..n), p (levels 0..n-1), u = p/gamma.

    y_tilde = (B^(2) kron M^{1/2}) y and p_tilde = ((B^(2))^T kron M^{1/2}) p
    (eqn:main_system; M = I for finite differences).
    """
    n, m = prob.n, prob.m
    b2 = B2(n, prob.theta).toarray()
    yt = mass_power(prob, x[: n * m].reshape(n, m), -0.5) / np.sqrt(prob.gamma)
    pt = mass_power(prob, x[n * m:].reshape(n, m), -0.5)
    y = sla.solve_triangular(b2, yt, lower=True)
    p = sla.solve_triangular(b2.T, pt, lower=False)
    return y, p, p / prob.gamma


def solve(prob: Problem, f, g, y0, method: str, tol=1e-8, maxit=500, restart=30):
    kind, symmetric = METHODS[method]
    op = AllAtOnce(prob)
    gt, ft = rhs_tilde(prob, f, g, y0)
    b = transformed_rhs(prob, gt, ft, symmetric)
    P = FastPreconditioner(prob, kind)
    if symmetric:
        x, it, hist = krylov.minres(op.A, b, P.apply, tol=tol, maxit=maxit)
        res = np.linalg.norm(b - op.A(x)) / np.linalg.norm(b)
    else:
        x, it, hist = krylov.gmres(op.Ahat, b, P.apply, tol=tol, restart=restart, maxit=maxit)
        res = np.linalg.norm(b - op.Ahat(x)) / np.linalg.norm(b)
    y, p, u = recover(prob, x)
    return dict(x=x, b=b, y=y, p=p, u=u, iters=it, relres=res, hist=hist)


def direct_solve(prob: Problem, f, g, y0):
    """Sparse direct solve of A_tilde [y; p] = [g_tilde; f_tilde] (eqn:main_system_before)."""
    gt, ft = rhs_tilde(prob, f, g, y0)
    At = assemble_Atilde(prob).tocsc()
    sol = spla.spsolve(At, np.concatenate([gt.ravel(), ft.ravel()]))
    nm = prob.n * prob.m
    return sol[:nm].reshape(prob.n, prob.m), sol[nm:].reshape(prob.n, prob.m)


def e_h(prob: Problem, y, p, y_exact, p_exact) -> float:
    """Discrete L^inf_tau(L^2) error of eqn:error_measure.

    Max over the 2n time slices (y at t_1..t_n, p at t_0..t_{n-1}) of
    h^{dims/2} * ||slice error||_2.  y_exact, p_exact are (n+1, m) samples at
    t_0..t_n.
    """
    w = prob.h ** (prob.dims / 2)
    ey = np.linalg.norm(y - y_exact[1:], axis=1)
    ep = np.linalg.norm(p - p_exact[:-1], axis=1)
    return float(w * max(ey.max(), ep.max()))
