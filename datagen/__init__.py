"""Seeded synthetic inputs for the parabolic tracking problem.

This module is shared by the CPU oracle and by the GPU path's tests and
benchmarks.  It only *samples* given functions on the grid (source f, target g,
initial state y0, diffusion coefficient a at cell faces, and the manufactured
exact solutions of the paper's examples); it holds none of the method's
arithmetic (no discretisation, no transforms, no solves).

Grid convention (Section 4 protocol): h = 1/(M+1), interior nodes x_i = i*h,
i = 1..M in each of `dims` dimensions, tau = T/n, time levels t_k = k*tau,
k = 0..n.  Space-time arrays are returned with shape (n+1, M**dims), time
major, spatial index x1 fastest (row-major [x2][x1] in 2D).

Coefficient layout ("face arrays"): a(x) enters the finite-difference operator
through its values at cell-face midpoints.  In 1D this is one array of M+1
values at x = (i+1/2)h, i = 0..M.  In 2D it is the concatenation of
  ax: shape (M, M+1)   -- faces normal to x1, at ((i+1/2)h, j h), row j=1..M
  ay: shape (M+1, M)   -- faces normal to x2, at (i h, (j+1/2)h), row j=0..M
flattened row-major, total 2*M*(M+1) values.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "nodes", "times", "face_coefficients", "smooth_modes", "noise",
    "sinusoidal_a", "example1", "example2", "config_problem", "CONFIGS",
    "log_uniform_gamma",
]


def nodes(M: int) -> np.ndarray:
    """Interior node coordinates i/(M+1), i = 1..M."""
    return np.arange(1, M + 1, dtype=np.float64) / (M + 1)


def times(n: int, T: float) -> np.ndarray:
    """Time levels k*T/n, k = 0..n."""
    return np.arange(0, n + 1, dtype=np.float64) * (T / n)


def _mesh(dims: int, M: int):
    x = nodes(M)
    if dims == 1:
        return (x,)
    x2, x1 = np.meshgrid(x, x, indexing="ij")  # row = x2, column = x1
    return (x1.ravel(), x2.ravel())


def sample_space_time(func, dims: int, M: int, n: int, T: float) -> np.ndarray:
    """Evaluate func(t, *x) on all time levels and interior nodes -> (n+1, M**dims)."""
    xs = _mesh(dims, M)
    t = times(n, T)
    out = np.empty((n + 1, M ** dims), dtype=np.float64)
    for k in range(n + 1):
        out[k] = func(t[k], *xs)
    return out


def face_coefficients(afunc, dims: int, M: int) -> np.ndarray:
    """Sample a(x) at cell-face midpoints in the layout described in the module doc."""
    h = 1.0 / (M + 1)
    xf = (np.arange(0, M + 1, dtype=np.float64) + 0.5) * h  # face positions
    xn = nodes(M)
    if dims == 1:
        return np.ascontiguousarray(afunc(xf), dtype=np.float64)
    # faces normal to x1: rows x2 = node j, columns x1 = face i
    X2, X1 = np.meshgrid(xn, xf, indexing="ij")
    ax = afunc(X1, X2)
    # faces normal to x2: rows x2 = face j, columns x1 = node i
    Y2, Y1 = np.meshgrid(xf, xn, indexing="ij")
    ay = afunc(Y1, Y2)
    return np.ascontiguousarray(np.concatenate([ax.ravel(), ay.ravel()]), dtype=np.float64)


def smooth_modes(seed: int, dims: int, M: int, n: int, T: float, nmodes: int = 4,
                 kmax: int = 8, jmax: int = 4) -> np.ndarray:
    """Sum of `nmodes` products sin(k1 pi x1)[sin(k2 pi x2)] cos(j pi t).

    Per mode: k ~ U{1..kmax} per dimension, j ~ U{0..jmax}, amplitude ~ N(0,1),
    drawn from numpy.random.default_rng(seed) in that order.
    """
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(nmodes):
        ks = [int(rng.integers(1, kmax + 1)) for _ in range(dims)]
        j = int(rng.integers(0, jmax + 1))
        amp = float(rng.standard_normal())
        modes.append((ks, j, amp))

    def func(t, *xs):
        acc = np.zeros_like(xs[0])
        for ks, j, amp in modes:
            term = amp * np.cos(j * np.pi * t) * np.ones_like(xs[0])
            for k, x in zip(ks, xs):
                term = term * np.sin(k * np.pi * x)
            acc = acc + term
        return acc

    return sample_space_time(func, dims, M, n, T)


def noise(seed: int, shape, sigma: float) -> np.ndarray:
    """IID N(0, sigma^2) values per node and time level."""
    rng = np.random.default_rng(seed)
    return sigma * rng.standard_normal(shape)


def sinusoidal_a(dims: int, M: int) -> np.ndarray:
    """a(x) = 1 + 0.5 sin(2 pi x1) sin(2 pi x2) (1D: 1 + 0.5 sin(2 pi x)) at faces."""
    if dims == 1:
        return face_coefficients(lambda x: 1.0 + 0.5 * np.sin(2 * np.pi * x), 1, M)
    return face_coefficients(
        lambda x1, x2: 1.0 + 0.5 * np.sin(2 * np.pi * x1) * np.sin(2 * np.pi * x2), 2, M)


def example1(M: int, n: int, T: float = 1.0):
    """The paper's Example 1 (2D, a = 1, Section 4): f, g, y0 and exact y, p.

    f = (2 pi^2 - 1) e^{-t} sin(pi x1) sin(pi x2), g = e^{-t} sin(pi x1) sin(pi x2),
    exact y = g, p = 0.  Returns dict of (n+1, m) arrays plus y0 (m,).
    """
    s = lambda t, x1, x2: np.exp(-t) * np.sin(np.pi * x1) * np.sin(np.pi * x2)
    g = sample_space_time(s, 2, M, n, T)
    f = (2 * np.pi ** 2 - 1) * g
    y = g.copy()
    p = np.zeros_like(g)
    return dict(f=f, g=g, y0=y[0].copy(), y_exact=y, p_exact=p, a_face=None)


def example2(M: int, n: int, gamma: float, T: float = 1.0):
    """The paper's Example 2 (2D, a = 1e-5 sin(pi x1 x2), Section 4).

    The printed f contains a factor "x(1-2x_2)" that is read as x_1(1-2x_2),
    the term the manufactured solution y = e^{-t} x1(1-x1) x2(1-x2),
    p = gamma sin(pi t) sin(pi x1) sin(pi x2) produces.
    """
    c = 1e-5
    pi = np.pi

    def f(t, x1, x2):
        return (-np.sin(pi * t) * np.sin(pi * x1) * np.sin(pi * x2)
                + np.exp(-t) * x1 * (1 - x1) * (2 * c * np.sin(pi * x1 * x2)
                                                 - x2 * (1 - x2)
                                                 - c * pi * np.cos(pi * x1 * x2) * x1 * (1 - 2 * x2))
                + np.exp(-t) * x2 * (1 - x2) * (2 * c * np.sin(pi * x1 * x2)
                                                 - c * pi * np.cos(pi * x1 * x2) * x2 * (1 - 2 * x1)))

    def g(t, x1, x2):
        return (-gamma * pi * np.cos(pi * t) * np.sin(pi * x1) * np.sin(pi * x2)
                + np.exp(-t) * x1 * (1 - x1) * x2 * (1 - x2)
                - c * gamma * pi ** 2 * np.sin(pi * t) * (
                    -2 * np.sin(pi * x1 * x2) * np.sin(pi * x1) * np.sin(pi * x2)
                    + np.cos(pi * x1 * x2) * (x1 * np.sin(pi * x1) * np.cos(pi * x2)
                                              + x2 * np.cos(pi * x1) * np.sin(pi * x2))))

    yex = lambda t, x1, x2: np.exp(-t) * x1 * (1 - x1) * x2 * (1 - x2)
    pex = lambda t, x1, x2: gamma * np.sin(pi * t) * np.sin(pi * x1) * np.sin(pi * x2)
    F = sample_space_time(f, 2, M, n, T)
    G = sample_space_time(g, 2, M, n, T)
    Y = sample_space_time(yex, 2, M, n, T)
    P = sample_space_time(pex, 2, M, n, T)
    a_face = face_coefficients(lambda x1, x2: c * np.sin(pi * x1 * x2), 2, M)
    return dict(f=F, g=G, y0=Y[0].copy(), y_exact=Y, p_exact=P, a_face=a_face)


def example3(M: int, n: int, T: float = 1.0, kappa: float = 1e-3):
    """The paper's Example 3 (2D, homogeneous Neumann data, a = 1e-3, Section 4) on the
    M x M grid of nodes x_j = j/(M-1) that includes the boundary nodes:
    f = (8 pi^2 a - 1) e^{-t} cos(2 pi x1) cos(2 pi x2), g = e^{-t} cos(2 pi x1) cos(2 pi x2),
    exact y = g, p = 0."""
    x = np.arange(M, dtype=np.float64) / (M - 1)
    X2, X1 = np.meshgrid(x, x, indexing="ij")
    c = (np.cos(2 * np.pi * X1) * np.cos(2 * np.pi * X2)).ravel()
    t = times(n, T)
    g = np.exp(-t)[:, None] * c[None, :]
    f = (8 * np.pi ** 2 * kappa - 1) * g
    return dict(f=f, g=g, y0=g[0].copy(), y_exact=g.copy(), p_exact=np.zeros_like(g),
                kappa=kappa)


# Workload recipes.  Each returns the problem parameters and FP64 arrays that
# both the oracle and the GPU path consume unchanged.
CONFIGS = {
    # 1D heat control, BE, MINRES-|P_S|
    "heat1d_M63_n64": dict(dims=1, M=63, n=64, T=1.0, theta=1.0, gamma=1e-4,
                           zeta=np.pi, coeff="const", noise=0.0, f_zero=True,
                           method="minres_abs_ps"),
    # 2D heat control, CN, GMRES(30)-P_S with sine-diagonalised spatial solves
    "heat2d_M255_n256": dict(dims=2, M=255, n=256, T=1.0, theta=0.5, gamma=1e-4,
                             zeta=np.pi, coeff="const", noise=1e-3, f_zero=False,
                             method="gmres_ps"),
    # 2D variable coefficient, multigrid spatial solves
    "heat2d_var_M255_n256": dict(dims=2, M=255, n=256, T=1.0, theta=0.5, gamma=1e-4,
                                 zeta=np.pi, coeff="sin", noise=1e-3, f_zero=False,
                                 method="gmres_ps"),
    # 2D mixed precision large case
    "heat2d_M511_n512": dict(dims=2, M=511, n=512, T=1.0, theta=0.5, gamma=1e-4,
                             zeta=np.pi, coeff="const", noise=1e-3, f_zero=False,
                             method="gmres_ps"),
}


def config_problem(dims: int, M: int, n: int, T: float = 1.0, seed: int = 0,
                   noise_sigma: float = 0.0, f_zero: bool = False,
                   coeff: str = "const", y0_zero: bool = True) -> dict:
    """Seeded synthetic data: g from seed, f from seed+1 (zero if f_zero), y0 = 0.

    Optional N(0, noise_sigma^2) noise on g (seed+2) and f (seed+3).
    coeff: "const" (a = 1, returns a_face=None) or "sin" (sinusoidal_a).
    """
    g = smooth_modes(seed, dims, M, n, T)
    f = np.zeros_like(g) if f_zero else smooth_modes(seed + 1, dims, M, n, T)
    if noise_sigma > 0:
        g = g + noise(seed + 2, g.shape, noise_sigma)
        if not f_zero:
            f = f + noise(seed + 3, f.shape, noise_sigma)
    y0 = np.zeros(M ** dims) if y0_zero else smooth_modes(seed + 4, dims, M, 0 + 1, T)[0]
    a_face = None if coeff == "const" else sinusoidal_a(dims, M)
    return dict(f=np.ascontiguousarray(f), g=np.ascontiguousarray(g), y0=y0, a_face=a_face)


def log_uniform_gamma(seed: int, lo: float = -8.0, hi: float = -2.0) -> float:
    """gamma = 10^U(lo, hi) drawn from default_rng(seed + 1000) (its own stream, so the
    data of the same seed does not change)."""
    return float(10.0 ** np.random.default_rng(seed + 1000).uniform(lo, hi))


def random_vector(seed: int, size: int) -> np.ndarray:
    """Standard normal FP64 vector (operator parity inputs)."""
    return np.random.default_rng(seed).standard_normal(size)
