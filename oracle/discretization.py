"""All-at-once discretisation (paper Section 1), FP64, scipy.sparse.

Notation follows the paper: M interior points per dimension, m = M**dims
spatial unknowns, h = 1/(M+1), n time steps, tau = T/n, alpha = tau/sqrt(gamma)
(eqn:matrix_A), theta in [1/2, 1] (theta = 1 backward Euler, 1/2 Crank-Nicolson).
Finite differences (disc = "fd"): mass matrix M_m = I, stiffness K_m = -L_m where
L_m is the (variable-coefficient) five-point Laplacian with homogeneous Dirichlet
data.  Finite elements (disc = "fem", a = 1): M_m and K_m are the consistent mass
and stiffness matrices of continuous piecewise-linear (1D) / bilinear (2D)
elements on the same grid; the system is the same with M_m in place of I
(eqn:matrix_A_before) and K_m -> M_m^{-1/2} K_m M_m^{-1/2} after the change of
variables (eqn:main_system).
Homogeneous Neumann data (bc = "neumann", Example 3, finite differences, constant
coefficient kappa): M nodes per dimension including both boundary nodes,
x_j = j h, h = 1/(M-1); the boundary rows use a mirrored ghost node, so K_m is not
symmetric, and the same K_m appears in the state and the adjoint block rows of
eqn:matrix_A_before (the system is then not symmetric: GMRES-P_S only).

Vectors are time major: a block vector [v^(1); ...; v^(n)] is an (n, m) array,
spatial index x1 fastest.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla


@dataclass
class Problem:
    dims: int
    M: int
    n: int
    T: float = 1.0
    theta: float = 1.0
    gamma: float = 1e-4
    zeta: float = np.pi
    a_face: Optional[np.ndarray] = None  # None => a == 1
    s2_remedy: float = 1.0
    disc: str = "fd"                       # "fd" or "fem"
    bc: str = "dirichlet"                  # "dirichlet" or "neumann"
    kappa: float = 1.0                     # constant a when a_face is None

    def __post_init__(self):
        if self.dims not in (1, 2):
            raise ValueError("dims must be 1 or 2")
        if self.disc not in ("fd", "fem"):
            raise ValueError("disc must be fd or fem")
        if self.bc not in ("dirichlet", "neumann"):
            raise ValueError("bc must be dirichlet or neumann")
        if self.disc == "fem" and self.a_face is not None:
            raise ValueError("the finite element form is built for a = 1")
        if self.a_face is not None and self.kappa != 1.0:
            raise ValueError("a variable coefficient carries its own scale (kappa = 1)")
        if not self.kappa > 0:
            raise ValueError("kappa must be positive")
        if self.bc == "neumann" and (self.disc != "fd" or self.a_face is not None or self.M < 2):
            raise ValueError("the Neumann form is finite differences with constant a, M >= 2")
        if not (0.5 <= self.theta <= 1.0):
            raise ValueError("theta must lie in [1/2, 1] (Section 1)")
        if self.gamma <= 0:
            raise ValueError("gamma must be positive")

    @property
    def h(self):
        return 1.0 / (self.M - 1) if self.bc == "neumann" else 1.0 / (self.M + 1)

    @property
    def m(self):
        return self.M ** self.dims

    @property
    def tau(self):
        return self.T / self.n

    @property
    def alpha(self):
        return self.tau / np.sqrt(self.gamma)


def stiffness(dims: int, M: int, a_face: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """K = -L_h: conservative five-point (three-point in 1D) finite differences.

    (K u)_P = sum over the faces f of P of a_f (u_P - u_nb(f)) / h^2, with
    u = 0 at boundary neighbours (homogeneous Dirichlet, eqn:heat).  a_f is the
    coefficient at the face midpoint (a = 1 when a_face is None).  Face layout
    as in datagen: 1D (M+1,); 2D ax (M, M+1) then ay (M+1, M).
    """
    h2 = (1.0 / (M + 1)) ** 2
    rows, cols, vals = [], [], []
    if dims == 1:
        a = np.ones(M + 1) if a_face is None else np.asarray(a_face, dtype=np.float64)
        assert a.shape == (M + 1,)
        for i in range(M):  # node x_{i+1}; left face a[i], right face a[i+1]
            diag = (a[i] + a[i + 1]) / h2
            rows.append(i); cols.append(i); vals.append(diag)
            if i > 0:
                rows.append(i); cols.append(i - 1); vals.append(-a[i] / h2)
            if i < M - 1:
                rows.append(i); cols.append(i + 1); vals.append(-a[i + 1] / h2)
        return sp.csr_matrix((vals, (rows, cols)), shape=(M, M))
    if a_face is None:
        ax = np.ones((M, M + 1))
        ay = np.ones((M + 1, M))
    else:
        a_face = np.asarray(a_face, dtype=np.float64)
        assert a_face.shape == (2 * M * (M + 1),)
        ax = a_face[: M * (M + 1)].reshape(M, M + 1)
        ay = a_face[M * (M + 1):].reshape(M + 1, M)
    idx = lambda i, j: j * M + i  # i = x1 index 0..M-1, j = x2 index 0..M-1
    for j in range(M):
        for i in range(M):
            P = idx(i, j)
            aw, ae = ax[j, i], ax[j, i + 1]      # west/east faces
            as_, an = ay[j, i], ay[j + 1, i]     # south/north faces
            rows.append(P); cols.append(P); vals.append((aw + ae + as_ + an) / h2)
            if i > 0:
                rows.append(P); cols.append(idx(i - 1, j)); vals.append(-aw / h2)
            if i < M - 1:
                rows.append(P); cols.append(idx(i + 1, j)); vals.append(-ae / h2)
            if j > 0:
                rows.append(P); cols.append(idx(i, j - 1)); vals.append(-as_ / h2)
            if j < M - 1:
                rows.append(P); cols.append(idx(i, j + 1)); vals.append(-an / h2)
    return sp.csr_matrix((vals, (rows, cols)), shape=(M * M, M * M))


def stiffness_neumann(dims: int, M: int, kappa: float = 1.0) -> sp.csr_matrix:
    """kappa times minus the three-point (1D) / five-point (2D) Laplacian on the M nodes
    x_j = j h, h = 1/(M-1), of a uniform grid that includes both boundary nodes, with
    homogeneous Neumann data imposed by a mirrored ghost node (u_{-1} = u_1,
    u_M = u_{M-2}): (K1 u)_0 = 2(u_0 - u_1)/h^2, (K1 u)_{M-1} = 2(u_{M-1} - u_{M-2})/h^2,
    interior rows (2 u_j - u_{j-1} - u_{j+1})/h^2.  2D: K1 along x1 plus K1 along x2."""
    h2 = (1.0 / (M - 1)) ** 2
    main = 2.0 * np.ones(M)
    lo = -np.ones(M - 1)
    up = -np.ones(M - 1)
    up[0] = -2.0          # row 0: the ghost u_{-1} = u_1 doubles the east weight
    lo[-1] = -2.0         # row M-1: the ghost u_M = u_{M-2} doubles the west weight
    K1 = sp.diags([main, lo, up], [0, -1, 1]) * (kappa / h2)
    if dims == 1:
        return K1.tocsr()
    I = sp.identity(M)
    return (sp.kron(I, K1) + sp.kron(K1, I)).tocsr()


def fem_matrices(dims: int, M: int):
    """(M_m, K_m) of continuous piecewise-linear (1D) or bilinear (2D) Lagrange elements
    on the uniform grid with interior nodes x_i = i h, h = 1/(M+1), a = 1, homogeneous
    Dirichlet data.  Element integrals of the hat functions:
    1D mass h/6 [1 4 1], stiffness 1/h [-1 2 -1]; the bilinear basis is the tensor
    product, so M = M1 kron M1 and K = K1 kron M1 + M1 kron K1 (x2 index outer)."""
    h = 1.0 / (M + 1)
    e = np.ones(M)
    M1 = sp.diags([4.0 * e, e[:-1], e[:-1]], [0, -1, 1]) * (h / 6.0)
    K1 = sp.diags([2.0 * e, -e[:-1], -e[:-1]], [0, -1, 1]) / h
    if dims == 1:
        return M1.tocsr(), K1.tocsr()
    return sp.kron(M1, M1).tocsr(), (sp.kron(K1, M1) + sp.kron(M1, K1)).tocsr()


def mass_stiffness(prob: "Problem"):
    """(M_m, K_m) of the problem's discretisation (Section 1)."""
    if prob.bc == "neumann":
        return sp.identity(prob.m, format="csr"), stiffness_neumann(prob.dims, prob.M, prob.kappa)
    if prob.disc == "fem":
        Mm, K = fem_matrices(prob.dims, prob.M)
        return Mm, K * prob.kappa
    return sp.identity(prob.m, format="csr"), stiffness(prob.dims, prob.M, prob.a_face) * prob.kappa


def mass_power(prob: "Problem", X: np.ndarray, power: float) -> np.ndarray:
    """Rows of X times M_m^power (power = +-1/2 in the change of variables of
    eqn:main_system).  M_m = I for finite differences; for the bilinear elements with
    a = 1 the orthonormal sine basis U (dense) diagonalises the 1D mass matrix,
    U M1 U = diag(h/3 (2 + cos(j pi h))), so M_m^power = (U kron U) diag(...)^power (U kron U)."""
    if prob.disc == "fd":
        return X
    M, h = prob.M, prob.h
    i = np.arange(1, M + 1)
    U = np.sqrt(2.0 / (M + 1)) * np.sin(np.outer(i, i) * np.pi / (M + 1))
    m1 = (h / 3.0) * (2.0 + np.cos(i * np.pi * h))
    shp = X.shape
    if prob.dims == 1:
        Y = X.reshape(-1, M) @ U.T
        Y = Y * m1 ** power
        return (Y @ U.T).reshape(shp)
    Y = X.reshape(-1, M, M) @ U.T          # along x1
    Y = np.matmul(U, Y)                    # along x2
    Y = Y * (np.outer(m1, m1) ** power)[None, :, :]
    Y = Y @ U.T
    Y = np.matmul(U, Y)
    return Y.reshape(shp)


def B1(n: int) -> sp.csr_matrix:
    """B_n^(1): unit lower bidiagonal, 1 on the diagonal, -1 below (Section 1)."""
    return sp.diags([np.ones(n), -np.ones(n - 1)], [0, -1], format="csr")


def B2(n: int, theta: float) -> sp.csr_matrix:
    """B_n^(2): theta on the diagonal, 1 - theta below (Section 1)."""
    return sp.diags([theta * np.ones(n), (1 - theta) * np.ones(n - 1)], [0, -1], format="csr")


def Bn_closed_form(n: int, theta: float) -> np.ndarray:
    """B_n = B^(1) (B^(2))^{-1} from its printed entries (Section 1, after eqn:matrix_T).

    Lower triangular Toeplitz: 1/theta on the diagonal, -1/theta^2 on the first
    subdiagonal and -(theta-1)^{k-1}/theta^{k+1} on the k-th subdiagonal, k >= 2.
    """
    col = np.zeros(n)
    col[0] = 1.0 / theta
    for k in range(1, n):
        col[k] = -((theta - 1.0) ** (k - 1)) / theta ** (k + 1)
    return sla.toeplitz(col, np.zeros(n))


def assemble_Atilde(prob: Problem) -> sp.csr_matrix:
    """The 2nm x 2nm matrix of eqn:matrix_A_before with M_m = I, K_m = K."""
    n, m, tau, th, gam = prob.n, prob.m, prob.tau, prob.theta, prob.gamma
    Mm, K = mass_stiffness(prob)
    b1, b2 = B1(n), B2(n, th)
    A11 = tau * sp.kron(b2, Mm)
    A12 = sp.kron(b1.T, Mm) + tau * sp.kron(b2.T, K)
    A21 = sp.kron(b1, Mm) + tau * sp.kron(b2, K)
    A22 = -(tau / gam) * sp.kron(b2.T, Mm)
    return sp.bmat([[A11, A12], [A21, A22]], format="csr")


class AllAtOnce:
    """Matrix-free applies of A_tilde, A (symmetric) and A_hat (nonsymmetric).

    A_tilde [y; p] uses the Kronecker identity (B kron C) vec(X) = vec(B X C^T)
    for time-major (n, m) arrays X; tests pin it against assemble_Atilde.
    A and A_hat are reached from A_tilde by the change of variables of
    eqn:main_system: x1 = sqrt(gamma) B^(2) y, x2 = (B^(2))^T p, second block
    row scaled by sqrt(gamma); A_hat is A with its block rows swapped
    (eqn:matrix_A_hat).
    """

    def __init__(self, prob: Problem):
        self.prob = prob
        self.Mm, self.K = mass_stiffness(prob)
        n = prob.n
        self.b1 = B1(n).toarray()
        self.b2 = B2(n, prob.theta).toarray()

    def Atilde(self, y: np.ndarray, p: np.ndarray):
        """Return the two block rows of A_tilde [y; p] for (n, m) arrays y, p."""
        pr, K, Mm = self.prob, self.K, self.Mm
        tau, gam = pr.tau, pr.gamma
        b1, b2 = self.b1, self.b2
        KY = (K @ y.T).T  # I_n kron K applied to y
        KP = (K @ p.T).T
        MY = (Mm @ y.T).T
        MP = (Mm @ p.T).T
        r1 = tau * (b2 @ MY) + b1.T @ MP + tau * (b2.T @ KP)
        r2 = b1 @ MY + tau * (b2 @ KY) - (tau / gam) * (b2.T @ MP)
        return r1, r2

    def to_yp(self, x1: np.ndarray, x2: np.ndarray):
        """[x1; x2] = [sqrt(gamma) y_tilde; p_tilde] -> (y, p), with
        y_tilde = (B^(2) kron M^{1/2}) y and p_tilde = ((B^(2))^T kron M^{1/2}) p."""
        g = np.sqrt(self.prob.gamma)
        y = sla.solve_triangular(self.b2, mass_power(self.prob, x1, -0.5) / g, lower=True)
        p = sla.solve_triangular(self.b2.T, mass_power(self.prob, x2, -0.5), lower=False)
        return y, p

    def A(self, x: np.ndarray) -> np.ndarray:
        """Symmetric operator of eqn:matrix_A applied to a flat 2nm vector: the change of
        variables of eqn:main_system around A_tilde (rows scaled by M^{-1/2})."""
        n, m = self.prob.n, self.prob.m
        x1 = x[: n * m].reshape(n, m)
        x2 = x[n * m:].reshape(n, m)
        y, p = self.to_yp(x1, x2)
        r1, r2 = self.Atilde(y, p)
        r1 = mass_power(self.prob, r1, -0.5)
        r2 = mass_power(self.prob, r2, -0.5)
        return np.concatenate([r1.ravel(), np.sqrt(self.prob.gamma) * r2.ravel()])

    def Ahat(self, x: np.ndarray) -> np.ndarray:
        """Nonsymmetric operator of eqn:matrix_A_hat (block rows of A swapped)."""
        nm = self.prob.n * self.prob.m
        r = self.A(x)
        return np.concatenate([r[nm:], r[:nm]])


def rhs_tilde(prob: Problem, f: np.ndarray, g: np.ndarray, y0: np.ndarray):
    """f_tilde and g_tilde of Section 1 (M_m = I) from samples at t_0..t_n.

    f, g: (n+1, m) arrays at time levels 0..n; y0: (m,).  Returns (g_t, f_t),
    each (n, m).
    """
    n, tau, th = prob.n, prob.tau, prob.theta
    Mm, K = mass_stiffness(prob)
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    y0 = np.asarray(y0, dtype=np.float64)
    ft = np.empty((n, prob.m))
    gt = np.empty((n, prob.m))
    for k in range(1, n + 1):  # block row k uses levels k-1 and k
        ft[k - 1] = Mm @ (th * tau * f[k] + (1 - th) * tau * f[k - 1])
        gt[k - 1] = tau * (Mm @ (th * g[k - 1] + (1 - th) * g[k]))
    ft[0] += Mm @ y0 - (1 - th) * tau * (K @ y0)
    gt[0] -= tau * (1 - th) * (Mm @ y0)
    return gt, ft


def transformed_rhs(prob: Problem, gt: np.ndarray, ft: np.ndarray, symmetric: bool) -> np.ndarray:
    """[g; sqrt(gamma) f] (eqn:main_system) or [sqrt(gamma) f; g] (eqn:main_system_nonsym),
    f = (I kron M^{-1/2}) f_tilde, g = (I kron M^{-1/2}) g_tilde."""
    sg = np.sqrt(prob.gamma)
    ft = mass_power(prob, ft, -0.5)
    gt = mass_power(prob, gt, -0.5)
    if symmetric:
        return np.concatenate([gt.ravel(), sg * ft.ravel()])
    return np.concatenate([sg * ft.ravel(), gt.ravel()])
