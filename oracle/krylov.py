"""Textbook Krylov solvers in FP64 for the oracle (Section 4 protocol: zero
initial guess, stopping tolerance on the relative residual).

The paper runs MATLAB's built-in `minres` and `gmres` without stating the norm
of its stopping test.  The oracle reads the tolerance as a bound on the TRUE
relative residual ||b - A x_k||_2 / ||b||_2, evaluated explicitly with the
operator after every iteration.

* minres: preconditioned MINRES (Lanczos three-term recurrence in the
  P^{-1} inner product, Givens QR of the tridiagonal matrix, short
  recurrence for the search directions) for symmetric A and symmetric
  positive definite P.
* gmres: restarted GMRES(k), right preconditioned, storing the
  preconditioned basis Z (flexible form, so x = x0 + Z y exactly), Arnoldi
  with classical Gram-Schmidt applied twice; the small least-squares problem
  min ||beta e1 - H y|| is solved with numpy.linalg.lstsq at every step.
"""
from __future__ import annotations

import numpy as np


def minres(A, b, Pinv, tol=1e-8, maxit=1000, x0=None):
    """Returns (x, iters, relres_history)."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    hist = []
    if nb == 0:
        return x, 0, [0.0]
    r = b - A(x)
    rel = np.linalg.norm(r) / nb
    hist.append(rel)
    if rel <= tol:
        return x, 0, hist
    v_prev = np.zeros_like(b)
    v = r
    z = Pinv(v)
    gam = np.sqrt(float(np.dot(z, v)))
    gam_prev = 1.0
    eta = gam
    s_prev, s = 0.0, 0.0
    c_prev, c = 1.0, 1.0
    w_prev = np.zeros_like(b)
    w = np.zeros_like(b)
    for it in range(1, maxit + 1):
        z = z / gam
        Az = A(z)
        delta = float(np.dot(Az, z))
        v_new = Az - (delta / gam) * v - (gam / gam_prev) * v_prev
        z_new = Pinv(v_new)
        gam_new = np.sqrt(max(float(np.dot(z_new, v_new)), 0.0))
        a0 = c * delta - c_prev * s * gam
        a1 = np.hypot(a0, gam_new)
        a2 = s * delta + c_prev * c * gam
        a3 = s_prev * gam
        c_new, s_new = a0 / a1, gam_new / a1
        w_new = (z - a3 * w_prev - a2 * w) / a1
        x = x + c_new * eta * w_new
        eta = -s_new * eta
        rel = np.linalg.norm(b - A(x)) / nb
        hist.append(rel)
        if rel <= tol or gam_new == 0.0:
            return x, it, hist
        v_prev, v = v, v_new
        z = z_new
        gam_prev, gam = gam, gam_new
        s_prev, s = s, s_new
        c_prev, c = c, c_new
        w_prev, w = w, w_new
    return x, maxit, hist


def gmres(A, b, Pinv, tol=1e-8, restart=30, maxit=1000, x0=None):
    """Right-preconditioned restarted GMRES with CGS2.  Returns (x, iters, hist)."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    hist = []
    if nb == 0:
        return x, 0, [0.0]
    total = 0
    r = b - A(x)
    rel = np.linalg.norm(r) / nb
    hist.append(rel)
    if rel <= tol:
        return x, 0, hist
    while total < maxit:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), dtype=b.dtype)
        xj = x
        for j in range(restart):
            z = Pinv(V[j])
            Z.append(z)
            w = A(z)
            Vm = np.array(V)
            h1 = Vm.conj() @ w
            w = w - Vm.T @ h1
            h2 = Vm.conj() @ w
            w = w - Vm.T @ h2
            H[: j + 1, j] = h1 + h2
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            e1 = np.zeros(j + 2, dtype=b.dtype)
            e1[0] = beta
            y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
            xj = x + np.array(Z).T @ y
            total += 1
            r = b - A(xj)
            rel = np.linalg.norm(r) / nb
            hist.append(rel)
            if rel <= tol or hn == 0.0 or total >= maxit:
                return xj, total, hist
            V.append(w / hn)
        x = xj
    return x, total, hist
