"""The preconditioners P_S (eqn:matrix_P_GMRES), |P_S| (eqn:matrix_P) and
P_MS (eqn:matrix_P_MS), plus the ideal |A| (eqn:abs_ideal_matrix_H).

Two forms:

* dense_*: the matrices themselves, built from their definitions with dense
  FP64 linear algebra (matrix square roots by Hermitian eigendecomposition).
  Only for tiny n, m.
* apply_*_inv: the three-step application of Section 3.4: (1) the time
  transform Phi kron I on both block rows, (2) independent spatial problems
  per time frequency, (3) the inverse transform.  Step (1)/(3) use the dense
  O(n^2) matrix Phi of circulant.transform.  Step (2) uses the dense sine
  basis when a = 1, and a sparse LU of each frequency's shifted operator
  otherwise.  Both block rows use the same Phi (the (2,2) block of the
  printed unitary carries a spurious adjoint; with the same transform in both
  blocks the off-diagonal alpha*I blocks are preserved, and S_n^* is
  diagonalised by Phi with conjugated eigenvalues because |omega| = 1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import circulant, spatial
from .discretization import Problem, stiffness, AllAtOnce, mass_stiffness


# ----------------------------------------------------------------------------
# dense definitions (tiny sizes)
# ----------------------------------------------------------------------------

def _herm_sqrt(H: np.ndarray) -> np.ndarray:
    H = 0.5 * (H + H.conj().T)
    w, V = np.linalg.eigh(H)
    w = np.clip(w, 0.0, None)
    return (V * np.sqrt(w)) @ V.conj().T


def dense_khat(prob: Problem) -> np.ndarray:
    """The spatial operator of the transformed system, M_m^{-1/2} K_m M_m^{-1/2}
    (eqn:matrix_A; -L_m for finite differences), with the inverse square root of the
    mass matrix from a dense symmetric eigendecomposition."""
    Mm, K = mass_stiffness(prob)
    if prob.disc == "fd":
        return K.toarray()
    w, V = np.linalg.eigh(Mm.toarray())
    Mis = (V / np.sqrt(w)) @ V.T
    return Mis @ K.toarray() @ Mis


def dense_calS(prob: Problem) -> np.ndarray:
    """S = S_n kron I_m + tau I_n kron (-L_m) (eqn:matrix_S)."""
    S = circulant.Sn(prob.n, prob.theta, prob.zeta, prob.s2_remedy)
    K = dense_khat(prob)
    return np.kron(S, np.eye(prob.m)) + prob.tau * np.kron(np.eye(prob.n), K)


def dense_PS(prob: Problem) -> np.ndarray:
    """P_S = [[S, -alpha I], [alpha I, S_n^* kron I + tau I kron K]]: the time factor B_n of
    the two block rows replaced by S_n and its adjoint; the spatial operator is the one of
    A_hat's blocks (for a symmetric K the (2,2) block is S^*)."""
    S = dense_calS(prob)
    Sn = circulant.Sn(prob.n, prob.theta, prob.zeta, prob.s2_remedy)
    K = dense_khat(prob)
    S2 = np.kron(Sn.conj().T, np.eye(prob.m)) + prob.tau * np.kron(np.eye(prob.n), K)
    a = prob.alpha
    I = np.eye(S.shape[0])
    return np.block([[S, -a * I], [a * I, S2]])


def dense_absPS(prob: Problem) -> np.ndarray:
    """|P_S| = sqrt(P_S^* P_S)."""
    P = dense_PS(prob)
    return _herm_sqrt(P.conj().T @ P)


def dense_PMS(prob: Problem) -> np.ndarray:
    """P_MS: sqrt(S_n^* S_n + alpha^2) kron I + tau I kron (-L) (and S S^* below)."""
    S = circulant.Sn(prob.n, prob.theta, prob.zeta, prob.s2_remedy)
    K = dense_khat(prob)
    a2 = prob.alpha ** 2
    In, Im = np.eye(prob.n), np.eye(prob.m)
    top = np.kron(_herm_sqrt(S.conj().T @ S + a2 * In), Im) + prob.tau * np.kron(In, K)
    bot = np.kron(_herm_sqrt(S @ S.conj().T + a2 * In), Im) + prob.tau * np.kron(In, K)
    Z = np.zeros_like(top)
    return np.block([[top, Z], [Z, bot]])


def dense_A(prob: Problem) -> np.ndarray:
    """The symmetric all-at-once matrix A, column by column through AllAtOnce.A."""
    op = AllAtOnce(prob)
    N = 2 * prob.n * prob.m
    E = np.eye(N)
    return np.column_stack([op.A(E[:, j]) for j in range(N)])


def dense_Ahat(prob: Problem) -> np.ndarray:
    op = AllAtOnce(prob)
    N = 2 * prob.n * prob.m
    E = np.eye(N)
    return np.column_stack([op.Ahat(E[:, j]) for j in range(N)])


def dense_absA(prob: Problem) -> np.ndarray:
    """|A| = sqrt(A^2) (eqn:abs_ideal_matrix_H)."""
    A = dense_A(prob)
    return _herm_sqrt(A @ A)


# ----------------------------------------------------------------------------
# three-step applies (config sizes)
# ----------------------------------------------------------------------------

class FastPreconditioner:
    """Three-step P^{-1} v for kind in {"ps", "abs_ps", "pms"}."""

    def __init__(self, prob: Problem, kind: str):
        if kind not in ("ps", "abs_ps", "pms"):
            raise ValueError(kind)
        if kind == "abs_ps" and prob.a_face is not None:
            raise ValueError("|P_S| needs a fast-diagonalisable -L (a = 1)")
        if kind != "ps" and prob.bc == "neumann":
            raise ValueError("the Neumann system is not symmetric: P_S (GMRES) only")
        self.prob, self.kind = prob, kind
        n = prob.n
        self.Phi = circulant.transform(n, prob.zeta)
        self.Phiinv = circulant.inverse_transform(n, prob.zeta)
        _, _, self.lam = circulant.eigen_tables(n, prob.theta, prob.zeta, prob.s2_remedy)
        self.K = mass_stiffness(prob)[1].tocsc()
        self._lu = {}

    # step 2 for one frequency l (variable a), spatial data v1, v2 (complex m-vectors)
    def _solve_frequency(self, l: int, v1: np.ndarray, v2: np.ndarray):
        pr = self.prob
        lam, tau, a = self.lam[l], pr.tau, pr.alpha
        m = pr.m
        # variable coefficient: sparse direct solves of the shifted systems
        if l not in self._lu:
            I = sp.identity(m, format="csc", dtype=np.complex128)
            K = self.K.astype(np.complex128)
            if self.kind == "pms":
                sig = np.sqrt(abs(lam) ** 2 + a * a)
                self._lu[l] = spla.splu((sig * I + tau * K).tocsc())
            else:  # "ps": the full 2m x 2m block of this frequency
                blk = sp.bmat([[lam * I + tau * K, -a * I],
                               [a * I, np.conj(lam) * I + tau * K]], format="csc")
                self._lu[l] = spla.splu(blk)
        lu = self._lu[l]
        if self.kind == "pms":
            return lu.solve(v1), lu.solve(v2)
        w = lu.solve(np.concatenate([v1, v2]))
        return w[:m], w[m:]

    def apply(self, v: np.ndarray, return_complex: bool = False) -> np.ndarray:
        pr = self.prob
        n, m = pr.n, pr.m
        V1 = v[: n * m].reshape(n, m).astype(np.complex128)
        V2 = v[n * m:].reshape(n, m).astype(np.complex128)
        H1 = self.Phi @ V1                    # step 1
        H2 = self.Phi @ V2
        W1 = np.empty_like(H1)
        W2 = np.empty_like(H2)
        if pr.a_face is None:                 # step 2, all frequencies at once
            neu = pr.bc == "neumann"
            if neu:
                mu = spatial.neumann_eigenvalues(pr.dims, pr.M, pr.kappa)
                T1 = spatial.cosine_transform(pr.dims, pr.M, H1, inverse=True)
                T2 = spatial.cosine_transform(pr.dims, pr.M, H2, inverse=True)
            else:
                mu = pr.kappa * (spatial.fem_eigenvalues(pr.dims, pr.M) if pr.disc == "fem"
                                 else spatial.eigenvalues(pr.dims, pr.M))
                T1 = spatial.sine_transform(pr.dims, pr.M, H1)
                T2 = spatial.sine_transform(pr.dims, pr.M, H2)
            Lam = self.lam[:, None] + pr.tau * mu[None, :]
            a = pr.alpha
            if self.kind == "abs_ps":
                s = 1.0 / np.sqrt(np.abs(Lam) ** 2 + a * a)
                T1, T2 = s * T1, s * T2
            elif self.kind == "pms":
                s = 1.0 / (np.sqrt(np.abs(self.lam) ** 2 + a * a)[:, None] + pr.tau * mu[None, :])
                T1, T2 = s * T1, s * T2
            else:
                det = np.abs(Lam) ** 2 + a * a
                T1, T2 = (np.conj(Lam) * T1 + a * T2) / det, (-a * T1 + Lam * T2) / det
            if neu:
                W1 = spatial.cosine_transform(pr.dims, pr.M, T1, inverse=False)
                W2 = spatial.cosine_transform(pr.dims, pr.M, T2, inverse=False)
            else:
                W1 = spatial.sine_transform(pr.dims, pr.M, T1)
                W2 = spatial.sine_transform(pr.dims, pr.M, T2)
        else:
            for l in range(n):
                W1[l], W2[l] = self._solve_frequency(l, H1[l], H2[l])
        X1 = self.Phiinv @ W1                 # step 3
        X2 = self.Phiinv @ W2
        out = np.concatenate([X1.ravel(), X2.ravel()])
        return out if return_complex else out.real.copy()
