"""Small dense solvers of the eigensolver (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``rayleigh_ritz`` -- the generalized eigenproblem H~ v = lambda S~ v of the
  LOBPCG subspace (Alg. lobpcg_block, Eq. for the coefficients alpha, beta,
  gamma) and of the inverse-iteration clusters (Alg. block_inverse_iteration).
* ``minres`` -- the local symmetric (possibly indefinite) solver used inside
  ALS (Sec. II.C.3), after Paige and Saunders: Lanczos tridiagonalisation with
  the least-squares problem solved by Givens rotations.
* ``lanczos_lowest`` -- Lanczos with full reorthogonalisation, for exact
  references on small spaces.
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np


def rayleigh_ritz(H: np.ndarray, S: np.ndarray, nev: int, drop_tol: float = 1e-12):
    """Lowest ``nev`` Ritz pairs of (H, S).

    1. Cholesky S = L L^T; if a pivot falls below drop_tol * max diag(S), use
       SVQB instead: S = U Sigma U^T, keep sigma > drop_tol * sigma_max,
       B = U_r Sigma_r^{-1/2}.  Otherwise B = L^{-T}.
    2. C = B^T H B; C = Y Lambda Y^T; V = B Y (so V^T S V = I).
    3. Ascending eigenvalues; each column of V signed so that its entry of
       largest magnitude is positive.
    Returns (evals[nev], V[m, nev], rank).
    """
    H = 0.5 * (H + H.T)
    S = 0.5 * (S + S.T)
    m = H.shape[0]
    dmax = float(np.max(np.diag(S)))
    use_chol = True
    try:
        L = np.linalg.cholesky(S)
        if np.min(np.diag(L) ** 2) <= drop_tol * dmax:
            use_chol = False
    except np.linalg.LinAlgError:
        use_chol = False
    if use_chol:
        B = np.linalg.inv(L).T
        rank = m
    else:
        sig, U = np.linalg.eigh(S)
        keep = sig > drop_tol * np.max(sig)
        B = U[:, keep] / np.sqrt(sig[keep])[None, :]
        rank = int(np.sum(keep))
    C = B.T @ H @ B
    C = 0.5 * (C + C.T)
    lam, Y = np.linalg.eigh(C)
    V = B @ Y
    nev = min(nev, V.shape[1])
    lam, V = lam[:nev], V[:, :nev]
    for j in range(nev):
        i = int(np.argmax(np.abs(V[:, j])))
        if V[i, j] < 0:
            V[:, j] = -V[:, j]
    return lam, V, rank


def minres(apply: Callable[[np.ndarray], np.ndarray], b: np.ndarray, x0: np.ndarray,
           rtol: float, maxiter: int) -> Tuple[np.ndarray, int, float]:
    """Solve A x = b for symmetric A (Paige-Saunders MINRES), warm-started.

    Stops when the residual norm estimate |phibar| <= rtol * ||b|| or after
    ``maxiter`` Lanczos steps, or at a Lanczos breakdown.  Returns
    (x, iterations, residual-norm estimate).
    """
    x = x0.astype(np.float64).copy()
    r = b - apply(x)
    beta1 = float(np.linalg.norm(r))
    bnorm = float(np.linalg.norm(b))
    tol = rtol * bnorm
    if beta1 <= tol or beta1 == 0.0:
        return x, 0, beta1
    v_prev = np.zeros_like(x)
    v = r / beta1
    beta = 0.0            # beta_k: coupling of v_{k-1} and v_k (0 for k = 1)
    c1, s1 = 1.0, 0.0     # rotation G_{k-2}
    c2, s2 = 1.0, 0.0     # rotation G_{k-1}
    d_prev = np.zeros_like(x)
    d_pprev = np.zeros_like(x)
    phibar = beta1
    it = 0
    for it in range(1, maxiter + 1):
        p = apply(v)
        alpha = float(np.vdot(v, p))
        p = p - alpha * v - beta * v_prev
        beta_next = float(np.linalg.norm(p))
        # previous rotations on the new column (beta_k, alpha_k, beta_{k+1})
        eps = s1 * beta
        dbar = c1 * beta
        delta = c2 * dbar + s2 * alpha
        gbar = -s2 * dbar + c2 * alpha
        gamma = float(np.hypot(gbar, beta_next))
        if gamma == 0.0:
            break
        c, s = gbar / gamma, beta_next / gamma
        tau = c * phibar
        phibar = -s * phibar
        d = (v - delta * d_prev - eps * d_pprev) / gamma
        x = x + tau * d
        d_pprev, d_prev = d_prev, d
        c1, s1, c2, s2 = c2, s2, c, s
        if abs(phibar) <= tol or beta_next == 0.0:
            break
        v_prev, v = v, p / beta_next
        beta = beta_next
    return x, it, abs(phibar)


def lanczos_lowest(apply: Callable[[np.ndarray], np.ndarray], n: int, nev: int, seed: int = 0,
                   maxdim: int = 400, tol: float = 1e-11) -> np.ndarray:
    """Lowest ``nev`` eigenvalues of a symmetric operator of dimension n by
    Lanczos with full reorthogonalisation (restart-free, grows to maxdim)."""
    rng = np.random.default_rng(seed)
    q = rng.normal(size=n)
    Q = [q / np.linalg.norm(q)]
    alphas, betas = [], []
    prev = None
    for j in range(min(maxdim, n)):
        w = apply(Q[-1])
        a = float(Q[-1] @ w)
        alphas.append(a)
        Qm = np.array(Q)
        for _ in range(2):
            w = w - Qm.T @ (Qm @ w)
        bnext = float(np.linalg.norm(w))
        T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
        ev = np.linalg.eigvalsh(T)[:nev]
        if prev is not None and len(ev) == nev and np.max(np.abs(ev - prev)) < tol * max(1.0, np.max(np.abs(ev))):
            return ev
        prev = ev if len(ev) == nev else None
        if bnext < 1e-14:
            break
        betas.append(bnext)
        Q.append(w / bnext)
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) + np.diag(betas[:len(alphas) - 1], -1)
    return np.linalg.eigvalsh(T)[:nev]
