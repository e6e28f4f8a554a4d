"""Tree tensor network states: gauge, environments, H_eff (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (real arithmetic throughout: every Hamiltonian here is real
symmetric, so all conjugations are identities).

* N(u) = [parent, children in id order] (no parent at the root).
* State tensor A_u has legs [a_{N(u)}, p]; TTNO tensor W_u has legs
  [w_{N(u)}, p_out, q_in] (Eq. ttns, Eq. ttno).  Auxiliary nodes have a
  physical leg of dimension 1.
* Environment of the directed edge u->v between bra state i and ket state j
  (the shaded blocks of Fig. variational / Fig. als):
      E^{ij}_{u->v}[b, w, a] = sum A^i_u[b_N, p] W_u[w_N, p, q] A^j_u[a_N, q]
                               prod_{c in N(u)\\v} E^{ij}_{c->u}[b_c, w_c, a_c]
  with the bra bond b, operator bond w and ket bond a on the edge (u, v).
  op=None means the identity operator (W = delta_pq, every w of dimension 1).
* H_eff at node u (Sec. II.C.2-3): with the orthogonality centre of the bra
  and ket at u,
      Y[b_N, p] = sum W[w_N, p, q] X[a_N, q] prod_{c in N(u)} E_{c->u}[b_c, w_c, a_c]
                  - s X[b_N, p].
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# Pairwise contraction order picked greedily by numpy; the intermediate-size
# cap is lifted so numpy does not fall back to one nested loop over all
# indices (the order of summation does not change the definitions below).
_EINSUM = ("greedy", 2 ** 40)


# ---------------------------------------------------------------- tree helpers

def nbrs(tree, u) -> List[int]:
    return tree.neighbours(u)


def leg_of(tree, u, v) -> int:
    """Position of the leg toward neighbour v in node u's tensors."""
    return nbrs(tree, u).index(v)


def identity_op(tree, u) -> np.ndarray:
    d = tree.phys[u]
    k = len(nbrs(tree, u))
    return np.eye(d).reshape((1,) * k + (d, d))


def path_next(tree, u, c) -> int:
    """Neighbour of u on the path from u to c (u != c)."""
    if c in tree.subtree(u):
        for ch in tree.children(u):
            if c in tree.subtree(ch):
                return ch
    return tree.parent[u]


def euler_tour(tree) -> List[int]:
    """Depth-first Euler tour from the root (node sequence, root first and last)."""
    out = []

    def rec(u):
        out.append(u)
        for c in tree.children(u):
            rec(c)
            out.append(u)

    rec(tree.root)
    return out


# ---------------------------------------------------------------- gauge (K6)

def qr_split(A: np.ndarray, leg: int) -> Tuple[np.ndarray, np.ndarray]:
    """Reshape A with ``leg`` last into [rest, D_e], Householder QR (numpy /
    LAPACK) with the signs fixed so that diag(R) >= 0 (Sec. II.A.1, splitting
    a tensor by QR).  Returns (Q reshaped back into A's leg order, R)."""
    T = np.moveaxis(A, leg, -1)
    sh = T.shape
    Q, R = np.linalg.qr(T.reshape(-1, sh[-1]))
    sg = np.where(np.diag(R) < 0, -1.0, 1.0)
    Q = Q * sg[None, :]
    R = sg[:, None] * R
    Qt = np.moveaxis(Q.reshape(sh[:-1] + (Q.shape[1],)), -1, leg)
    return Qt, R


def absorb(A: np.ndarray, leg: int, R: np.ndarray) -> np.ndarray:
    """A[.., leg=old, ..] -> sum_old R[new, old] A[.., old, ..]."""
    return np.moveaxis(np.tensordot(R, A, axes=([1], [leg])), 0, leg)


def move_centre(tree, state: List[np.ndarray], u: int, v: int) -> None:
    """Move the orthogonality centre from u to its neighbour v (in place)."""
    Q, R = qr_split(state[u], leg_of(tree, u, v))
    state[u] = Q
    state[v] = absorb(state[v], leg_of(tree, v, u), R)


def canonicalize(tree, state: List[np.ndarray], centre: int) -> List[np.ndarray]:
    """Bring a state to canonical form with its orthogonality centre at
    ``centre`` (every other tensor an isometry toward the centre)."""
    st = [a.copy() for a in state]

    def rec(u, frm):
        for w in nbrs(tree, u):
            if w != frm:
                rec(w, u)
        if frm is not None:
            move_centre(tree, st, u, frm)

    rec(centre, None)
    return st


def norm_centre(state, centre) -> float:
    return float(np.linalg.norm(state[centre]))


# ---------------------------------------------------------------- K1 / K1'

def env_update(tree, u, v, bra: np.ndarray, W: Optional[np.ndarray], ket: np.ndarray,
               envs_in: Dict[int, np.ndarray]) -> np.ndarray:
    """E_{u->v}[b, w, a] from node u's bra, operator and ket tensors and the
    incoming environments E_{c->u} for c in N(u) \\ {v} (keyed by c)."""
    N = nbrs(tree, u)
    k = len(N)
    if W is None:
        W = identity_op(tree, u)
    B = list(range(0, k))
    Wl = list(range(k, 2 * k))
    A = list(range(2 * k, 3 * k))
    p, q = 3 * k, 3 * k + 1
    args = [bra, B + [p], W, Wl + [p, q], ket, A + [q]]
    iv = N.index(v)
    for i, c in enumerate(N):
        if c == v:
            continue
        args += [envs_in[c], [B[i], Wl[i], A[i]]]
    return np.einsum(*args, [B[iv], Wl[iv], A[iv]], optimize=_EINSUM)


def closure(tree, u, bra, W, ket, envs_in: Dict[int, np.ndarray]) -> float:
    """<bra|O|ket> closed at node u from all incoming environments."""
    N = nbrs(tree, u)
    k = len(N)
    if W is None:
        W = identity_op(tree, u)
    B = list(range(0, k))
    Wl = list(range(k, 2 * k))
    A = list(range(2 * k, 3 * k))
    p, q = 3 * k, 3 * k + 1
    args = [bra, B + [p], W, Wl + [p, q], ket, A + [q]]
    for i, c in enumerate(N):
        args += [envs_in[c], [B[i], Wl[i], A[i]]]
    return float(np.einsum(*args, [], optimize=_EINSUM))


def all_envs_toward(tree, root, bra, W, ket) -> Dict[Tuple[int, int], np.ndarray]:
    """Every environment E_{u->v} on edges pointing toward ``root``."""
    envs: Dict[Tuple[int, int], np.ndarray] = {}

    def rec(u, frm):
        for c in nbrs(tree, u):
            if c != frm:
                rec(c, u)
        if frm is not None:
            ein = {c: envs[(c, u)] for c in nbrs(tree, u) if c != frm}
            envs[(u, frm)] = env_update(tree, u, frm, bra[u], None if W is None else W[u], ket[u], ein)

    rec(root, None)
    return envs


def expectation(tree, bra, W, ket, at: Optional[int] = None) -> float:
    """<bra|O|ket> (O = TTNO W, or identity when W is None), closed at ``at``."""
    u = tree.root if at is None else at
    envs = all_envs_toward(tree, u, bra, W, ket)
    ein = {c: envs[(c, u)] for c in nbrs(tree, u)}
    return closure(tree, u, bra[u], None if W is None else W[u], ket[u], ein)


# ---------------------------------------------------------------- K2 / K3

def heff_apply(tree, u, W: Optional[np.ndarray], X: np.ndarray, envs_in: Dict[int, np.ndarray],
               shift: float = 0.0) -> np.ndarray:
    """Y = (H_eff - s) X at node u (K2); W None -> identity operator."""
    N = nbrs(tree, u)
    k = len(N)
    if W is None:
        W = identity_op(tree, u)
    B = list(range(0, k))
    Wl = list(range(k, 2 * k))
    A = list(range(2 * k, 3 * k))
    p, q = 3 * k, 3 * k + 1
    args = [W, Wl + [p, q], X, A + [q]]
    for i, c in enumerate(N):
        args += [envs_in[c], [B[i], Wl[i], A[i]]]
    Y = np.einsum(*args, B + [p], optimize=_EINSUM)
    if shift != 0.0:
        Y = Y - shift * X
    return Y


def heff_diag(tree, u, W, envs_in, shift: float = 0.0) -> np.ndarray:
    """diag[b_N, p] = sum_w W[w, p, p] prod_c E_c[b_c, w_c, b_c] - s  (K3)."""
    N = nbrs(tree, u)
    k = len(N)
    B = list(range(0, k))
    Wl = list(range(k, 2 * k))
    p = 2 * k
    Wd = np.einsum(W, Wl + [p, p], Wl + [p])
    args = [Wd, Wl + [p]]
    for i, c in enumerate(N):
        Ed = np.einsum(envs_in[c], [0, 1, 0], [0, 1])  # E[b, w, b]
        args += [Ed, [B[i], Wl[i]]]
    return np.einsum(*args, B + [p], optimize=_EINSUM) - shift


def heff_dense(tree, u, W, envs_in, shift=0.0) -> np.ndarray:
    """Explicit H_eff matrix (n_loc x n_loc) by applying K2 to unit vectors."""
    N = nbrs(tree, u)
    shape = tuple(envs_in[c].shape[2] for c in N) + (W.shape[-1],)
    n = int(np.prod(shape))
    H = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        H[:, i] = heff_apply(tree, u, W, e.reshape(shape), envs_in, shift).ravel()
    return H


# ---------------------------------------------------------------- K4

def gram(tree, states: Sequence[List[np.ndarray]], W) -> Tuple[np.ndarray, np.ndarray]:
    """H~_kl = <s_k|H|s_l>, S~_kl = <s_k|s_l> over the given states (upper
    triangle computed by full pair contractions, then mirrored)."""
    m = len(states)
    H = np.zeros((m, m))
    S = np.zeros((m, m))
    for a in range(m):
        for b in range(a, m):
            H[a, b] = H[b, a] = expectation(tree, states[a], W, states[b])
            S[a, b] = S[b, a] = expectation(tree, states[a], None, states[b])
    return H, S


# ---------------------------------------------------------------- dense embedding

def to_dense(tree, state) -> np.ndarray:
    """Full coefficient vector over modes 0..L-1 (tiny trees only)."""
    def rec(u):
        T = state[u]
        has_par = tree.parent[u] >= 0
        tags = (["par"] if has_par else []) + [("ch", c) for c in tree.children(u)] + [("m", tree.mode[u])]
        for c in tree.children(u):
            Tc, tc = rec(c)
            pos = tags.index(("ch", c))
            T = np.tensordot(T, Tc, axes=([pos], [0]))
            tags = tags[:pos] + tags[pos + 1:] + tc[1:]
        return T, tags

    T, tags = rec(tree.root)
    keep = [i for i, t in enumerate(tags) if t[0] == "m" and t[1] >= 0]
    aux = [i for i, t in enumerate(tags) if t[0] == "m" and t[1] < 0]
    T = T.reshape([T.shape[i] if i not in aux else 1 for i in range(T.ndim)])
    T = np.squeeze(T, axis=tuple(aux)) if aux else T
    modes = [tags[i][1] for i in keep]
    order = np.argsort(modes)
    return np.transpose(T, order).ravel()


def isometry_at(tree, state, u) -> np.ndarray:
    """P_u: the explicit map from node u's local vector to the full space
    (columns = full vectors), valid when the state's centre is u."""
    shape = state[u].shape
    n = int(np.prod(shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        st = list(state)
        st[u] = e.reshape(shape)
        cols.append(to_dense(tree, st))
    return np.stack(cols, axis=1)
