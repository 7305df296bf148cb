"""omega-circulant time factors (Section 1, eqn:matrix_S and the definitions of
S_n^(1), S_n^(2) that follow it), dense FP64.

The paper prints an eigendecomposition of S_n^(j) (eqn:decompositiob_S12) whose
transform and eigenvalue ordering do not reproduce S_n^(1) as written; the set
of eigenvalues it lists is right.  The oracle therefore does not use the
printed factorisation.  It builds the matrices entry by entry, takes the
transform Phi = F D (D = diag(omega^{k/n}) = diag(e^{i zeta k/n}), F the
unnormalised DFT with kernel e^{-2 pi i k l/n}), and reads the eigenvalues off
the similarity Phi S Phi^{-1} itself.  Tests check that this similarity is
diagonal and that its diagonal equals the closed form of the lemma on
S_n^* + S_n (Section 3.3).
"""
from __future__ import annotations

import numpy as np


def omega_circulant(first_col: np.ndarray, omega: complex) -> np.ndarray:
    """n x n omega-circulant: C[j,k] = c[j-k] (j >= k), omega * c[n+j-k] (j < k)."""
    c = np.asarray(first_col, dtype=np.complex128)
    n = c.size
    C = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        for k in range(n):
            C[j, k] = c[j - k] if j >= k else omega * c[n + j - k]
    return C


def S1(n: int, zeta: float) -> np.ndarray:
    """S_n^(1): 1 on the diagonal, -1 below, -omega in the top-right corner."""
    c = np.zeros(n)
    c[0], c[1] = 1.0, -1.0
    return omega_circulant(c, np.exp(1j * zeta))


def S2(n: int, theta: float, zeta: float) -> np.ndarray:
    """S_n^(2): theta on the diagonal, 1-theta below, omega(1-theta) top-right."""
    c = np.zeros(n)
    c[0], c[1] = theta, 1.0 - theta
    return omega_circulant(c, np.exp(1j * zeta))


def transform(n: int, zeta: float) -> np.ndarray:
    """Phi[l, k] = e^{-2 pi i k l / n} e^{i zeta k / n}: the O(n^2) time transform."""
    k = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(k, k) / n)
    D = np.exp(1j * zeta * k / n)
    return F * D[None, :]


def inverse_transform(n: int, zeta: float) -> np.ndarray:
    """Phi^{-1} = D^{-1} F^{-1}: [k, l] = e^{-i zeta k/n} e^{2 pi i k l/n} / n."""
    k = np.arange(n)
    Finv = np.exp(2j * np.pi * np.outer(k, k) / n) / n
    Dinv = np.exp(-1j * zeta * k / n)
    return Dinv[:, None] * Finv


def similarity_diagonal(C: np.ndarray, zeta: float):
    """Return (diag, max |off-diagonal|) of Phi C Phi^{-1}."""
    n = C.shape[0]
    X = transform(n, zeta) @ C @ inverse_transform(n, zeta)
    d = np.diag(X).copy()
    off = X - np.diag(d)
    return d, float(np.max(np.abs(off))) if n > 1 else 0.0


def eigen_tables(n: int, theta: float, zeta: float, s2_remedy: float = 1.0):
    """Eigenvalue tables (lambda1, lambda2_remedied, lambda) in transform order.

    lambda^(j)_l = (Phi S^(j) Phi^{-1})_{ll}.  A zero eigenvalue of S^(2)
    (possible for theta = 1/2, e.g. zeta = 0 with n even or zeta = pi with n
    odd) is replaced by the nonzero real `s2_remedy` (remark after
    eqn:decompositiob_S12); s2_remedy = 0 raises.
    lambda = lambda1 / lambda2 are the eigenvalues of S_n = S^(1) (S^(2))^{-1}.
    """
    l1, _ = similarity_diagonal(S1(n, zeta), zeta)
    l2, _ = similarity_diagonal(S2(n, theta, zeta), zeta)
    sing = np.abs(l2) < 1e-12
    if np.any(sing):
        if s2_remedy == 0.0:
            raise ZeroDivisionError("S^(2) is singular and no remedy value was given")
        l2 = l2.copy()
        l2[sing] = s2_remedy
    return l1, l2, l1 / l2


def Sn(n: int, theta: float, zeta: float, s2_remedy: float = 1.0) -> np.ndarray:
    """S_n = S^(1) (S~^(2))^{-1} as a dense matrix (remedied S^(2) if singular)."""
    s1 = S1(n, zeta)
    s2 = S2(n, theta, zeta)
    _, l2, _ = eigen_tables(n, theta, zeta, s2_remedy)
    s2r = inverse_transform(n, zeta) @ np.diag(l2) @ transform(n, zeta)
    return s1 @ np.linalg.inv(s2r)


def lemma_eigenvalues(n: int, theta: float, zeta: float) -> np.ndarray:
    """Closed form of lambda_k(S_n), k = 0..n-1, from the lemma on S_n^* + S_n."""
    k = np.arange(n)
    e = np.exp(1j * (zeta + 2 * np.pi * k) / n)
    return (1 - e) / (theta + (1 - theta) * e)


def lemma_hermitian_part(n: int, theta: float, zeta: float) -> np.ndarray:
    """Closed form of lambda_k(S_n^* + S_n) from the same lemma."""
    k = np.arange(n)
    c = np.cos((zeta + 2 * np.pi * k) / n)
    return 2 * (2 * theta - 1) * (1 - c) / (theta ** 2 + (1 - theta) ** 2 + 2 * theta * (1 - theta) * c)
