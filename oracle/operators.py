"""Per-mode operator matrices (oracle; test infrastructure only).

Basis: the harmonic-oscillator functions |0>..|d-1> of each mode (finite basis
representation).  q = (a + a^dagger)/sqrt(2) in dimensionless normal
coordinates.  Powers q^n are the exact Galerkin projection: the top-left d x d
block of (Q_{d+n})^n, where Q_m is q in a basis of size m (q^n only couples
|k> to |k+-n>, so that block is exact).  The harmonic on-site operator
omega/2 (p^2 + q^2) is then diag(omega (n + 1/2)) exactly.

The Hermite DVR of the paper (Sec. III.A, kinetic matrix T_mn of Baye's
formula and q = diag of the Hermite roots) is provided as an alternative.
"""
from __future__ import annotations

import numpy as np


def ho_q(m: int) -> np.ndarray:
    """q in the HO basis of size m: <k-1|q|k> = <k|q|k-1> = sqrt(k/2)."""
    q = np.zeros((m, m))
    for k in range(1, m):
        q[k - 1, k] = q[k, k - 1] = np.sqrt(k / 2.0)
    return q


def ho_p2(m: int) -> np.ndarray:
    """Exact projection of p^2 onto |0>..|m-1> (built in size m+2)."""
    n = m + 2
    a = np.zeros((n, n))
    for k in range(1, n):
        a[k - 1, k] = np.sqrt(k)
    p = (a.T - a) / np.sqrt(2.0)  # p = i (a^dag - a)/sqrt2, real part of -i p
    p2 = -(p @ p)
    return p2[:m, :m]


def ho_qpow(d: int, n: int) -> np.ndarray:
    """Exact projection of q^n onto |0>..|d-1>."""
    if n == 0:
        return np.eye(d)
    Q = ho_q(d + n)
    return np.linalg.matrix_power(Q, n)[:d, :d]


def ho_number(d: int) -> np.ndarray:
    return np.diag(np.arange(d, dtype=np.float64))


def hermite_nodes(N: int) -> np.ndarray:
    """Roots of the Hermite polynomial H_N (physicists')."""
    x, _ = np.polynomial.hermite.hermgauss(N)
    return np.sort(x)


def dvr_kinetic(N: int) -> np.ndarray:
    """Baye's Hermite-DVR kinetic matrix (Sec. III.A): off-diagonal
    (-1)^(m-n) (2/(x_m-x_n)^2 - 1/2), diagonal (4N - 1 - 2 x_m^2)/6."""
    x = hermite_nodes(N)
    T = np.zeros((N, N))
    for m in range(N):
        for n in range(N):
            if m == n:
                T[m, n] = (4 * N - 1 - 2 * x[m] ** 2) / 6.0
            else:
                T[m, n] = (-1) ** (m - n) * (2.0 / (x[m] - x[n]) ** 2 - 0.5)
    return T


def mode_operators(d: int, omega: float, basis: str = "fbr"):
    """(onsite, qpow) for one mode: onsite = omega * n (the harmonic term with
    the zero-point energy omega/2 removed, i.e. shifted frame); qpow(k) = q^k."""
    if basis == "fbr":
        onsite = omega * ho_number(d)
        return onsite, (lambda k: ho_qpow(d, k))
    if basis == "dvr":
        x = hermite_nodes(d)
        onsite = 0.5 * omega * (dvr_kinetic(d) + np.diag(x ** 2)) - 0.5 * omega * np.eye(d)
        return onsite, (lambda k: np.diag(x ** k))
    raise ValueError(basis)
