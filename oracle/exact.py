"""Exact references for the eigensolver (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* Normal modes: for H = sum_i omega_i/2 (p_i^2 + q_i^2) + sum_{i<j} c_ij q_i q_j
  (Eq. coupled_harmonic_oscillator; exact levels are available analytically,
  Sec. III.A) write H = 1/2 p^T Omega p + 1/2 q^T K q with Omega = diag(omega),
  K = diag(omega) + C.  The substitution q = Omega^{1/2} y gives normal-mode
  frequencies Nu^2 = eig(diag(omega^2) + sqrt(omega_i omega_j) c_ij) and levels
  E = sum_k Nu_k (n_k + 1/2).
* The sum-of-products Hamiltonian applied to a dense vector through its
  Kronecker structure, one mode factor at a time (no TTNO involved).
"""
from __future__ import annotations

import heapq
from typing import List

import numpy as np

from .operators import mode_operators


def normal_mode_frequencies(model) -> np.ndarray:
    L = model.n_modes
    w = np.asarray(model.omega, dtype=np.float64)
    C = np.zeros((L, L))
    for mono, c in zip(model.monomials, model.coefs):
        if len(mono) == 2 and all(p == 1 for _, p in mono):
            (i, _), (j, _) = mono
            C[i, j] = C[j, i] = c
        elif any(p > 0 for _, p in mono):
            raise ValueError("normal modes need a purely quadratic model")
    A = np.diag(w ** 2) + np.sqrt(np.outer(w, w)) * C
    nu2 = np.linalg.eigvalsh(A)
    if np.min(nu2) <= 0:
        raise ValueError("unstable quadratic form")
    return np.sqrt(nu2)


def normal_mode_levels(model, k: int, shifted: bool = True) -> np.ndarray:
    """Lowest k levels of the quadratic model (shifted frame: minus sum omega/2)."""
    nu = normal_mode_frequencies(model)
    base = 0.5 * float(np.sum(nu))
    L = len(nu)
    heap = [(0.0, tuple([0] * L))]
    seen = {heap[0][1]}
    out: List[float] = []
    while len(out) < k:
        e, n = heapq.heappop(heap)
        out.append(e)
        for i in range(L):
            m = list(n)
            m[i] += 1
            m = tuple(m)
            if m not in seen:
                seen.add(m)
                heapq.heappush(heap, (e + nu[i], m))
    E = np.array(out) + base
    if shifted:
        E = E - model.zpe_harmonic
    return E


def sop_apply_dense(model, v: np.ndarray, basis: str = "fbr") -> np.ndarray:
    """H' v for the full tensor-product space (shifted frame), mode 0 slowest."""
    dims = list(model.dims)
    T = v.reshape(dims)
    ops = [mode_operators(d, float(w), basis) for d, w in zip(dims, model.omega)]
    out = np.zeros_like(T)

    def apply_mode(X, i, M):
        return np.moveaxis(np.tensordot(M, X, axes=([1], [i])), 0, i)

    for i in range(len(dims)):
        out += apply_mode(T, i, ops[i][0])
    for mono, c in zip(model.monomials, model.coefs):
        Y = T
        for i, p in mono:
            Y = apply_mode(Y, i, ops[i][1](p))
        out += c * Y
    return out.ravel()


def sop_dense_matrix(model, basis: str = "fbr") -> np.ndarray:
    n = int(np.prod(model.dims))
    H = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        H[:, i] = sop_apply_dense(model, e, basis)
    return H
