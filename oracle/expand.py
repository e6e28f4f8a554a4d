"""Bond expansion of a TTNS from the residual of the local target (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. II.C.2 (variational fitting, dynamic bond dimensions): after a local
solve the residual of the local system is formed, and where it is large a
rank-revealing QR of it supplies the directions by which the solution is
expanded.  Sec. III.B then raises the maximum bond dimension between the
LOBPCG stage (D = 12) and the inverse-iteration refinement (D = 20).  Here
both are one operation, applied once at that transition: every bond of x grows
to the prescribed size, x itself is kept exactly, and the new directions of
each bond are the leading pivots of a column-pivoted QR of the local residual
of H x -- the part of the locally assembled H x that the current basis of the
bond does not span.

Reading (the paper gives no formula): the local H x at node u is assembled
with the children legs in the already expanded bases and the parent leg left
open; that leg is probed with a Gaussian Khatri-Rao sketch of n columns
(the environments of <omega_l| H |x> from the parent side, exactly as in
successive randomized compression, Sec. II.C.1), and the rank-revealing QR
acts on the sketch.  The residual is the part of the sketch outside the span
of the current local basis Q_x of x: a Householder QR of [Q_x | S] whose first
columns (Q_x) are taken in order and whose remaining steps pivot over the
sketch columns (largest remaining norm, first in index order on ties) leaves
the current basis in front and orthonormal completions after it, orthogonal
to it even where the sketch has fewer independent directions than the growth.

Steps, leaves to root (children before parents):
1. sketch environments of <omega_l| H |x> on every edge (as SRC, step 1);
2. at each non-root node u with parent p:
   a. X_u = x_u with each child leg c mapped by B_c (the environment <y|x>
      of the expanded child, identity operator), the parent leg open:
      matricized [rest x D_u], QR (diag(R) >= 0) gives the basis Q_x;
   b. S_u[:, l] = node u's H and x tensors contracted with the children's
      <y|H|x> environments and the parent-side sketch environment l
      (the local sketch of H x, [rest x n]);
   c. Householder QR of [Q_x | S_u]: D_u unpivoted steps over Q_x, then
      P = D'_u - D_u steps pivoting over the sketch columns;
   d. the new directions are columns D_u .. D'_u - 1 of its Q (diag(R) >= 0);
   e. y_u = [Q_x, P] with parent leg D'_u; B_u = <y|x> and <y|H|x> are
      updated across the edge u -> p;
3. the root: y_root = x_root with each child leg mapped by B_c.
The result represents x exactly (the new directions carry zero weight) and is
canonical at the root.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from . import ttn
from .src import _post_order, sketch_envs


def _delta_env(D: int) -> np.ndarray:
    """Identity-operator environment that leaves a leg open: E[b, 1, a] = delta_ba."""
    return np.eye(D).reshape(D, 1, D)


def pivoted_completion(Q: np.ndarray, S: np.ndarray, grow: int, diag_out: list = None) -> np.ndarray:
    """Steps c-d: Householder QR of [Q | S] (Q: [m x D] orthonormal columns,
    taken first and unpivoted; then `grow` steps, each bringing forward the
    remaining column of largest norm below the diagonal, the first one on
    ties).  Returns columns D .. D + grow - 1 of the orthogonal factor, each
    signed so that its diagonal entry of R is >= 0."""
    A = np.concatenate([Q, S], axis=1).astype(np.float64)
    m, D = A.shape[0], Q.shape[1]
    K = D + grow
    if K > m:
        raise ValueError("more columns than rows")
    vs, diag = [], []
    for k in range(K):
        if k >= D:
            norms = [np.linalg.norm(A[k:, j]) for j in range(k, A.shape[1])]
            j = k + int(np.argmax(norms))  # argmax returns the first maximum
            A[:, [k, j]] = A[:, [j, k]]
        x = A[k:, k].copy()
        nx = np.linalg.norm(x)
        sg = 1.0 if x[0] >= 0 else -1.0
        v = x
        v[0] += sg * nx          # reflector H = I - 2 v v^T / (v^T v) maps x to -sg |x| e_1
        vv = float(v @ v)
        if vv > 0:
            A[k:, k:] -= np.outer(v, (2.0 / vv) * (v @ A[k:, k:]))
        vs.append((v, vv))
        diag.append(-sg * nx)
    if diag_out is not None:
        diag_out.extend(diag[D:])
    out = np.zeros((m, grow))
    for i, k in enumerate(range(D, K)):
        q = np.zeros(m)
        q[k] = 1.0
        for h in range(k, -1, -1):  # Q e_k = H_0 H_1 ... H_k e_k
            v, vv = vs[h]
            if vv > 0:
                q[h:] -= (2.0 / vv) * (v @ q[h:]) * v
        out[:, i] = q if diag[k] >= 0 else -q
    return out


def expand_bonds(tree, W, x, new_bonds: Sequence[int], omegas: Sequence[np.ndarray], n: int, info: dict = None):
    """x grown to new_bonds[u] on every edge (u, parent(u)) (new_bonds[u] >= x's
    bond).  omegas[u]: the d_u x n Gaussian test matrix of physical node u; n
    must be at least the largest growth.  Returns the expanded state y (canonical
    at the root, equal to x as a vector).  Where the residual sketch has fewer
    independent directions than the growth, the last completions are orthonormal
    but otherwise arbitrary (whatever the reflectors of the rank-deficient tail
    give); with `info`, info[u] = (D_u, r_u) records the number r_u of
    completions whose R diagonal exceeds 1e-8 of the sketch's norm -- the
    determined ones."""
    sk = sketch_envs(tree, W, x, omegas, n)  # 1.
    y: List[np.ndarray] = [None] * tree.n  # type: ignore[list-item]
    B: Dict[int, np.ndarray] = {}    # <y|x> across edge (u, parent(u)), [D'_u, 1, D_u]
    BH: Dict[int, np.ndarray] = {}   # <y|H|x> across edge (u, parent(u)), [D'_u, M_u, D_u]
    for u in _post_order(tree):
        p = tree.parent[u]
        ch = tree.children(u)
        if p < 0:  # 3.
            y[u] = ttn.heff_apply(tree, u, None, x[u], {c: B[c] for c in ch})
            continue
        Du = x[u].shape[0]  # the parent leg comes first
        grow = new_bonds[u] - Du
        if grow < 0 or grow > n:
            raise ValueError("new bond below the current one, or growth above the sketch size")
        # a. the local x with its parent leg open
        ein = {c: B[c] for c in ch}
        ein[p] = _delta_env(Du)
        Xu = ttn.heff_apply(tree, u, None, x[u], ein)              # [D_u, rest...]
        Qx, R = ttn.qr_split(Xu, 0)
        rest = int(np.prod(Xu.shape[1:]))
        Q = np.moveaxis(Qx, 0, -1).reshape(rest, Du)
        # b. the local sketch of H x
        cols = []
        for l in range(n):
            e2 = {c: BH[c] for c in ch}
            e2[p] = sk[l][(p, u)]
            cols.append(ttn.heff_apply(tree, u, W[u], x[u], e2)[0].ravel())
        S = np.stack(cols, axis=1)                                  # [rest, n]
        # c.-d. rank-revealing QR of the residual outside the current basis
        dg: list = []
        Yu = np.concatenate([Q, pivoted_completion(Q, S, grow, dg)], axis=1) if grow > 0 else Q
        if info is not None:
            info[u] = (Du, int(np.sum(np.abs(np.array(dg)) > 1e-8 * max(np.linalg.norm(S), 1e-300))))
        # e. the expanded node and the environments across (u, p)
        y[u] = np.moveaxis(Yu.reshape(Xu.shape[1:] + (Du + grow,)), -1, 0)
        B[u] = ttn.env_update(tree, u, p, y[u], None, x[u], {c: B[c] for c in ch})
        BH[u] = ttn.env_update(tree, u, p, y[u], W[u], x[u], {c: BH[c] for c in ch})
    return y
