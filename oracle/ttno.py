"""Sum-of-products Hamiltonian -> tree tensor network operator (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper builds its TTNO (Eq. ttno) from the sum-of-products form
(Eq. sum_of_tp) through a compressed state diagram (Sec. II.A.3).  Any exact
TTNO represents the same operator, so the oracle uses the plainest exact
construction and then removes redundant channels:

1. Naive automaton.  Across the edge between the subtree S of node u and the
   rest of the tree, every term is in one of three situations: none of its
   modes lie in S (channel "identity"), all of them do (channel "done", which
   carries the coefficient), or it is split, in which case the channel is the
   distinct partial product of its operators inside S.  Node tensors route
   these channels: identity -> identity, one child's "done" -> "done",
   children partials + the local factor -> the parent's partial (coefficient 1)
   or -> "done" (coefficient c_t) at the lowest node whose subtree holds the
   whole term.
2. Compression.  Orthogonalise toward the root with QR, then sweep down from
   the root with SVDs, keeping singular values above ``rel_tol`` times the
   largest one.  This yields the operator Schmidt rank on every edge.

Layout: ``W[u]`` has legs [w_parent, w_child1, ..., p_out, q_in] (no parent
leg at the root), children ordered by node id.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .operators import mode_operators

# Term = (coef, {mode: opkey}); opkey ("n",) on-site harmonic, ("q", k) q^k.


def model_terms(model):
    """The Hamiltonian in the ZPE-shifted frame: sum_i omega_i n_i + monomials."""
    terms = []
    for i in range(model.n_modes):
        terms.append((1.0, {i: ("n",)}))
    for mono, c in zip(model.monomials, model.coefs):
        terms.append((float(c), {m: ("q", p) for m, p in mono}))
    return terms


def _op_matrix(model, mode, key, basis):
    onsite, qpow = mode_operators(model.dims[mode], float(model.omega[mode]), basis)
    if key[0] == "n":
        return onsite
    return qpow(key[1])


def automaton_ttno(tree, model, basis: str = "fbr"):
    """Exact TTNO from the naive automaton (no compression)."""
    terms = model_terms(model)
    n = tree.n
    node_of_mode = {tree.mode[u]: u for u in range(n) if tree.mode[u] >= 0}
    subtree = [set(tree.subtree(u)) for u in range(n)]
    children = [tree.children(u) for u in range(n)]

    def label(t, u):
        """Channel of term t on the edge above u: 'I', 'done' or a partial."""
        inside = tuple(sorted((m, k) for m, k in t[1].items() if node_of_mode[m] in subtree[u]))
        if not inside:
            return "I"
        if len(inside) == len(t[1]):
            return "done"
        return inside

    # channel lists per edge (edge = child node id)
    chans: List[Dict] = [dict() for _ in range(n)]
    for u in range(n):
        if tree.parent[u] < 0:
            continue
        lab = {"I": 0, "done": 1}
        parts = sorted({label(t, u) for t in terms} - {"I", "done"})
        for p in parts:
            lab[p] = len(lab)
        chans[u] = lab

    def lowest_holder(t):
        nodes = [node_of_mode[m] for m in t[1]]
        u = nodes[0]
        while not all(x in subtree[u] for x in nodes):
            u = tree.parent[u]
        return u

    W = []
    for u in range(n):
        d = tree.phys[u]
        shape = []
        if tree.parent[u] >= 0:
            shape.append(len(chans[u]))
        shape += [len(chans[c]) for c in children[u]]
        shape += [d, d]
        Wu = np.zeros(shape)
        has_par = tree.parent[u] >= 0
        eye = np.eye(d)

        def put(par_ch, ch_children, op):
            idx = ([par_ch] if has_par else []) + list(ch_children)
            Wu[tuple(idx)] += op

        allI = [0] * len(children[u])
        if has_par:
            put(0, allI, eye)  # identity -> identity
        done_out = 1 if has_par else None
        for ci, c in enumerate(children[u]):  # a child's "done" passes up
            chs = list(allI)
            chs[ci] = 1
            if has_par:
                put(1, chs, eye)
            else:
                put(None, chs, eye)
        mymode = tree.mode[u]
        for t in terms:  # terms completed at u
            if lowest_holder(t) != u:
                continue
            chs = [chans[c][label(t, c)] for c in children[u]]
            op = _op_matrix(model, mymode, t[1][mymode], basis) if mymode in t[1] else eye
            put(done_out, chs, t[0] * op)
        if has_par:  # partials passing through u (each distinct partial once)
            for P, idx in chans[u].items():
                if P in ("I", "done"):
                    continue
                Pd = dict(P)
                chs = []
                for c in children[u]:
                    sub = tuple(sorted((m, k) for m, k in Pd.items() if node_of_mode[m] in subtree[c]))
                    chs.append(0 if not sub else chans[c][sub])
                op = _op_matrix(model, mymode, Pd[mymode], basis) if mymode in Pd else eye
                put(idx, chs, op)
        if not has_par:
            Wu = Wu  # root: legs [children..., p, q]
        W.append(Wu)
    return W


def _postorder(tree):
    out = []

    def rec(u):
        for c in tree.children(u):
            rec(c)
        out.append(u)

    rec(tree.root)
    return out


def _leg_of_child(tree, u, c):
    """Position of the leg toward child c in W[u]."""
    off = 1 if tree.parent[u] >= 0 else 0
    return off + tree.children(u).index(c)


def _absorb(T, leg, Mat):
    """Contract T's leg ``leg`` (dim old) with Mat[new, old] -> leg dim new."""
    T2 = np.tensordot(Mat, T, axes=([1], [leg]))  # new leg first
    return np.moveaxis(T2, 0, leg)


def compress_ttno(tree, W, rel_tol: float = 1e-13):
    """QR toward the root, then an SVD sweep down (see module doc)."""
    W = [w.copy() for w in W]
    root = tree.root
    # 1. orthogonalise every non-root tensor toward its parent
    for u in _postorder(tree):
        if u == root:
            continue
        Mpar = W[u].shape[0]
        rest = W[u].shape[1:]
        Mat = W[u].reshape(Mpar, -1).T
        Q, R = np.linalg.qr(Mat)
        W[u] = Q.T.reshape((Q.shape[1],) + rest)
        p = tree.parent[u]
        W[p] = _absorb(W[p], _leg_of_child(tree, p, u), R)

    # 2. truncating sweep down from the root, centre moving with the sweep
    def down(u):
        for c in tree.children(u):
            leg = _leg_of_child(tree, u, c)
            T = np.moveaxis(W[u], leg, -1)
            sh = T.shape
            U, s, Vt = np.linalg.svd(T.reshape(-1, sh[-1]), full_matrices=False)
            keep = int(np.sum(s > rel_tol * s[0])) if s.size and s[0] > 0 else 1
            keep = max(keep, 1)
            W[u] = np.moveaxis(U[:, :keep].reshape(sh[:-1] + (keep,)), -1, leg)
            W[c] = _absorb(W[c], 0, s[:keep, None] * Vt[:keep])
            down(c)
            Mpar = W[c].shape[0]
            rest = W[c].shape[1:]
            Q, R = np.linalg.qr(W[c].reshape(Mpar, -1).T)
            W[c] = Q.T.reshape((Q.shape[1],) + rest)
            W[u] = _absorb(W[u], leg, R)

    down(root)
    return W


def build_ttno(tree, model, basis: str = "fbr", compress: bool = True, rel_tol: float = 1e-13):
    """TTNO site tensors for ``model`` on ``tree`` (shifted frame, real FP64)."""
    W = automaton_ttno(tree, model, basis)
    if compress:
        W = compress_ttno(tree, W, rel_tol)
    return W


def ttno_bonds(tree, W) -> List[int]:
    """M_e for every edge (entry u = bond between u and its parent; 0 at root)."""
    return [W[u].shape[0] if tree.parent[u] >= 0 else 0 for u in range(tree.n)]


def ttno_to_dense(tree, W) -> np.ndarray:
    """Contract the whole TTNO to a dense matrix over modes 0..L-1 (row-major
    in mode order).  Only for tiny trees."""
    def rec(u):
        # returns (tensor with legs [w_parent?, P..., Q...], modes list)
        T = W[u]
        has_par = tree.parent[u] >= 0
        nch = len(tree.children(u))
        modes = [tree.mode[u]] if tree.mode[u] >= 0 else []
        # current: legs [par?, ch1..chm, p, q]; collapse aux p,q of dim 1
        if tree.mode[u] < 0:
            T = T[..., 0, 0]
            P, Q = [], []
        else:
            P, Q = [T.ndim - 2], [T.ndim - 1]
        for ci, c in enumerate(tree.children(u)):
            Tc, mc = rec(c)
            leg = (1 if has_par else 0) + ci
            # find current axis of that child leg: we always contract the
            # leading child leg remaining, which sits at position leg-ci
            pos = (1 if has_par else 0)
            T = np.tensordot(T, Tc, axes=([pos], [0]))
            # new axes: [par?, remaining ch..., own P/Q..., prev child P/Q..., Tc P..., Tc Q...]
            modes = modes + mc
        del nch
        return T, modes

    T, modes = rec(tree.root)
    # axes now: own p,q (if physical root) followed by each child's (P..., Q...)
    # rebuild an explicit ordering by re-deriving per-axis mode tags
    tags = _axis_tags(tree, tree.root)
    assert len(tags) == T.ndim
    L = len([m for m in tree.mode if m >= 0])
    order_p = [tags.index(("p", m)) for m in range(L)]
    order_q = [tags.index(("q", m)) for m in range(L)]
    T = np.transpose(T, order_p + order_q)
    dims = [T.shape[i] for i in range(L)]
    N = int(np.prod(dims))
    return T.reshape(N, N)


def _axis_tags(tree, u):
    """Axis tags of rec(u)'s output, mirroring ttno_to_dense's contraction order."""
    tags = []
    if tree.parent[u] >= 0:
        tags.append(("w", u))
    if tree.mode[u] >= 0:
        tags += [("p", tree.mode[u]), ("q", tree.mode[u])]
    for c in tree.children(u):
        tags += [t for t in _axis_tags(tree, c) if t[0] != "w"]
    return tags
