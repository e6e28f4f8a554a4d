"""Successive randomized compression (SRC) of a TTNO-TTNS product (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. II.C.1 (Eq. matrix random compression, Fig. random tensor, Fig. src):
the product y ~ H x of a TTNO H and a TTNS x is compressed to bond dimension
chi without forming the enlarged network.  The random test matrix is a
Khatri-Rao product: column l of Omega is the product vector
omega_l = (x)_j Omega^(j)[:, l] over the physical nodes j, Omega^(j) a
d_j x chi matrix drawn by the caller (passed in here).  So every sketch is a
contraction of <omega_l| H |x>, a network with a bond-one bra.

Steps, in the paper's order:
1. Sketch environments of <omega_l|H|x> for every edge, in both directions
   (K1 environments with the product bra omega_l).
2. From the leaves toward the root, at each non-root node i whose children
   are already compressed: the local sketch Y_i = A Omega, i.e. node i's
   tensors of H and x contracted with the compressed children (the B
   environments below) and with the sketch of everything outside subtree(i)
   (the environment parent(i) -> i of step 1), one column per l.  Its QR
   factorisation (Householder, diag(R) >= 0) gives the orthonormal Q_i, the
   new tensor at node i with chi columns on its parent leg.  When the node's
   local space has no more than chi dimensions, Q_i is the identity: the
   compressed node keeps the whole space, exactly.
3. B_{i -> parent(i)} = Q_i^T contracted with node i's H and x tensors and the
   children's B environments (the K1 environment <y|H|x> of the new tensor).
4. At the root everything left is contracted directly: y_root = node root's H
   and x tensors with the children's B environments.
The result is canonical with its orthogonality centre at the root.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import ttn


def _omega_state(tree, omegas: Sequence[np.ndarray], l: int) -> List[np.ndarray]:
    """Column l of the Khatri-Rao test matrix as a bond-one TTNS."""
    out = []
    for u in range(tree.n):
        shape = [1] * len(ttn.nbrs(tree, u))
        vec = omegas[u][:, l] if tree.phys[u] > 1 else np.ones(1)
        out.append(vec.reshape(shape + [tree.phys[u]]))
    return out


def _post_order(tree) -> List[int]:
    out = []

    def rec(u):
        for c in tree.children(u):
            rec(c)
        out.append(u)

    rec(tree.root)
    return out


def sketch_envs(tree, W, x, omegas: Sequence[np.ndarray], n: int) -> List[Dict[Tuple[int, int], np.ndarray]]:
    """Step 1: for every sketch column l < n, the environments of
    <omega_l| H |x> on every directed edge (toward the root, then away)."""
    sk: List[Dict[Tuple[int, int], np.ndarray]] = []
    for l in range(n):
        om = _omega_state(tree, omegas, l)
        envs: Dict[Tuple[int, int], np.ndarray] = {}
        for u in _post_order(tree):
            p = tree.parent[u]
            if p >= 0:
                ein = {c: envs[(c, u)] for c in ttn.nbrs(tree, u) if c != p}
                envs[(u, p)] = ttn.env_update(tree, u, p, om[u], W[u], x[u], ein)
        for u in reversed(_post_order(tree)):
            for c in tree.children(u):
                ein = {v: envs[(v, u)] for v in ttn.nbrs(tree, u) if v != c}
                envs[(u, c)] = ttn.env_update(tree, u, c, om[u], W[u], x[u], ein)
        sk.append(envs)
    return sk


def src_apply(tree, W, x, omegas: Sequence[np.ndarray], chi: int):
    """y ~ H x with bond dimension chi (Sec. II.C.1).  omegas[u] is the
    d_u x chi Gaussian test matrix of physical node u (ignored at auxiliary
    nodes).  Returns (y, bonds) with y canonical at the root and bonds[u] the
    dimension of edge (u, parent(u))."""
    # 1. all environments of <omega_l| H |x>
    sk = sketch_envs(tree, W, x, omegas, chi)
    # 2.-3. leaves to root
    y: List[np.ndarray] = [None] * tree.n  # type: ignore[list-item]
    B: Dict[int, np.ndarray] = {}           # B_{u -> parent(u)}[q, w, a]
    bonds = [0] * tree.n
    for u in _post_order(tree):
        p = tree.parent[u]
        ch = tree.children(u)
        if p < 0:
            # 4. root: direct contraction with the compressed children
            y[u] = ttn.heff_apply(tree, u, W[u], x[u], {c: B[c] for c in ch})
            continue
        cols = []
        for l in range(chi):
            ein = {c: B[c] for c in ch}
            ein[p] = sk[l][(p, u)]
            cols.append(ttn.heff_apply(tree, u, W[u], x[u], ein)[0].ravel())  # parent leg of the bra is 1
        Y = np.stack(cols, axis=1)  # [(children legs..., p), l]
        m = Y.shape[0]
        if m <= chi:
            Q = np.eye(m)
        else:
            Q, R = np.linalg.qr(Y)
            # the sign convention of the gauge moves: diag(R) >= 0
            s = np.sign(np.diag(R))
            s[s == 0] = 1.0
            Q = Q * s
        bonds[u] = Q.shape[1]
        legs = [y[c].shape[0] for c in ch] + [tree.phys[u]]
        y[u] = Q.T.reshape([Q.shape[1]] + legs)
        ein = {c: B[c] for c in ch}
        B[u] = ttn.env_update(tree, u, p, y[u], W[u], x[u], ein)
    return y, bonds
