"""Spatial eigenbasis of -L_h for a = 1 (Section 3.4, fast sine transform).

Textbook facts for the three-point / five-point Dirichlet Laplacian on a
uniform grid with h = 1/(M+1): the orthonormal sine matrix
U[i, j] = sqrt(2/(M+1)) sin(i j pi/(M+1)), i, j = 1..M, is symmetric and its
own inverse, and U (-L_h) U = diag(mu) with mu_j = 4 h^-2 sin^2(j pi h / 2)
(1D); in 2D the basis is U kron U with eigenvalues mu_j1 + mu_j2.

Homogeneous Neumann data on the M nodes x_j = j h, h = 1/(M-1) (both boundary nodes
included, mirrored ghost nodes): the cosine matrix C[j, k] = cos(j k pi/(M-1)),
j, k = 0..M-1, holds eigenvectors of the three-point operator K1 (its columns), with
eigenvalues 4 h^-2 sin^2(k pi h / 2); C is not orthogonal, and its inverse is
(2/(M-1)) W C W with W = diag(1/2, 1, ..., 1, 1/2) (the trapezoidal weights under which
the cosines are orthogonal).
"""
from __future__ import annotations

import numpy as np


def sine_matrix(M: int) -> np.ndarray:
    i = np.arange(1, M + 1)
    return np.sqrt(2.0 / (M + 1)) * np.sin(np.outer(i, i) * np.pi / (M + 1))


def laplacian_eigenvalues(M: int) -> np.ndarray:
    """mu_j, j = 1..M (1D)."""
    h = 1.0 / (M + 1)
    j = np.arange(1, M + 1)
    return 4.0 / h ** 2 * np.sin(j * np.pi * h / 2) ** 2


def eigenvalues(dims: int, M: int) -> np.ndarray:
    """Eigenvalues of -L_h in the order of the (x2, x1) row-major grid index."""
    mu = laplacian_eigenvalues(M)
    if dims == 1:
        return mu
    return (mu[:, None] + mu[None, :]).ravel()  # [j2][j1]


def sine_transform(dims: int, M: int, X: np.ndarray) -> np.ndarray:
    """Apply U (1D) or U kron U (2D) to every row of X (rows = spatial vectors).

    X has shape (..., M**dims); the transform is its own inverse.
    """
    U = sine_matrix(M)
    if dims == 1:
        return X @ U.T
    shp = X.shape
    Y = X.reshape(-1, M, M)            # [., x2, x1]
    Y = Y @ U.T                        # along x1
    Y = np.matmul(U, Y)                # along x2
    return Y.reshape(shp)


def fem_eigenvalues(dims: int, M: int) -> np.ndarray:
    """Eigenvalues of M_m^{-1/2} K_m M_m^{-1/2} for the linear / bilinear elements (a = 1):
    the sine basis diagonalises the 1D mass and stiffness matrices with
    m_j = h/3 (2 + cos(j pi h)) and k_j = 2/h (1 - cos(j pi h)), so in 1D mu_j = k_j/m_j and
    in 2D (k1 m2 + m1 k2)/(m1 m2) = mu_j1 + mu_j2, in the (x2, x1) row-major order."""
    h = 1.0 / (M + 1)
    j = np.arange(1, M + 1)
    mu = (2.0 / h) * (1.0 - np.cos(j * np.pi * h)) / ((h / 3.0) * (2.0 + np.cos(j * np.pi * h)))
    if dims == 1:
        return mu
    return (mu[:, None] + mu[None, :]).ravel()


def cosine_matrix(M: int) -> np.ndarray:
    k = np.arange(M)
    return np.cos(np.outer(k, k) * np.pi / (M - 1))


def cosine_inverse(M: int) -> np.ndarray:
    w = np.ones(M)
    w[0] = w[-1] = 0.5
    return (2.0 / (M - 1)) * (w[:, None] * cosine_matrix(M) * w[None, :])


def neumann_eigenvalues(dims: int, M: int, kappa: float = 1.0) -> np.ndarray:
    """Eigenvalues of the Neumann operator kappa K1 (1D) or kappa (K1 along x1 + K1 along
    x2) in the (x2, x1) row-major order of the cosine basis."""
    h = 1.0 / (M - 1)
    k = np.arange(M)
    mu = kappa * 4.0 / h ** 2 * np.sin(k * np.pi * h / 2) ** 2
    if dims == 1:
        return mu
    return (mu[:, None] + mu[None, :]).ravel()


def cosine_transform(dims: int, M: int, X: np.ndarray, inverse: bool) -> np.ndarray:
    """Rows of X (spatial vectors) times C^{-1} (inverse=True: into the cosine basis) or
    C (back to nodal values); 2D along x1 and x2."""
    A = cosine_inverse(M) if inverse else cosine_matrix(M)
    if dims == 1:
        return X @ A.T
    shp = X.shape
    Y = X.reshape(-1, M, M) @ A.T      # along x1
    Y = np.matmul(A, Y)                # along x2
    return Y.reshape(shp)
