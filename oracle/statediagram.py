"""TTNO construction from a state diagram with minimum vertex covers (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. II.A.3 builds the TTNO (Eq. ttno) of a sum-of-products Hamiltonian
(Eq. sum_of_tp) from a state diagram: across every edge the terms form a
bipartite graph between their parts on the two sides; a minimum vertex cover
of that graph gives the edge's channels (its bond dimension), and symbolic
Gaussian elimination places the coefficients so that every term is carried
exactly once.  The paper sketches the procedure; this is one reading of it,
written out:

Edges are treated leaves to root.  At the edge e above node v every current
item (a term, or a group of terms merged further down) is an edge of the
bipartite graph between
  * its left vertex: the descriptor of its part in subtree(v) -- its operator
    at v (or the identity) and the channel it uses on each child edge of v;
  * its right vertex: its operator string outside subtree(v).
A minimum vertex cover (Konig: from a maximum matching found by augmenting
paths, left vertices in order of first appearance) chooses the channels:
  * a covered left vertex is a channel that carries that descriptor with
    coefficient 1; its items keep their coefficients and right strings;
  * a covered right vertex R (with the left end uncovered) is a channel that
    carries the sum of coefficient x descriptor over its items -- they are
    merged into one item whose coefficient is 1 and whose operator is R from
    here on (the elimination: the coefficients are placed once, here).
An item merged at an edge outside subtree(v) must reach it through a
coefficient-free channel (its left vertex is forced into the cover):
otherwise two merged groups of different branches would multiply into cross
terms.  Channels are numbered: covered left vertices in order of first
appearance, then covered right vertices likewise.  The root sums every
remaining item with its coefficient.

Layout as oracle.ttno: W[u] has legs [w_parent, w_children..., p_out, q_in].
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np

from .ttno import _op_matrix, model_terms


def _post_order(tree) -> List[int]:
    out = []

    def rec(u):
        for c in tree.children(u):
            rec(c)
        out.append(u)

    rec(tree.root)
    return out


def min_vertex_cover(nl: int, nr: int, adj: List[List[int]], forced_left=()) -> Tuple[List[int], List[int]]:
    """Minimum vertex cover of a bipartite graph (left 0..nl-1, right
    0..nr-1, adj[l] = right neighbours in order) containing the forced left
    vertices: they are taken, their edges dropped, and the rest is covered by
    Konig's construction from a maximum matching (augmenting paths tried from
    each left vertex in order, neighbours in order).  Returns (left, right)
    vertex lists, ascending."""
    forced = set(forced_left)
    adj2 = [[] if l in forced else list(adj[l]) for l in range(nl)]
    match_l = [-1] * nl
    match_r = [-1] * nr
    for l0 in range(nl):
        if not adj2[l0]:
            continue
        # iterative augmenting-path search (depth first, neighbours in order)
        seen = [False] * nr
        stack = [(l0, 0)]
        path = []  # (l, r) tentative pairs along the search
        found = False
        while stack and not found:
            l, i = stack[-1]
            if i >= len(adj2[l]):
                stack.pop()
                if path:
                    path.pop()
                continue
            stack[-1] = (l, i + 1)
            r = adj2[l][i]
            if seen[r]:
                continue
            seen[r] = True
            path.append((l, r))
            if match_r[r] < 0:
                found = True
            else:
                stack.append((match_r[r], 0))
                continue
        if found:
            for l, r in path:
                match_l[l] = r
                match_r[r] = l
    # Konig: Z = vertices reachable from the unmatched left vertices by
    # alternating paths; cover = (L \\ Z) u (R n Z)
    visL = [False] * nl
    visR = [False] * nr
    stack = [l for l in range(nl) if match_l[l] < 0 and adj2[l]]
    for l in stack:
        visL[l] = True
    while stack:
        l = stack.pop()
        for r in adj2[l]:
            if not visR[r] and match_l[l] != r:
                visR[r] = True
                l2 = match_r[r]
                if l2 >= 0 and not visL[l2]:
                    visL[l2] = True
                    stack.append(l2)
    left = [l for l in range(nl) if l in forced or (adj2[l] and not visL[l])]
    right = [r for r in range(nr) if visR[r]]
    return left, right


def state_diagram_ttno(tree, model, basis: str = "fbr"):
    """Site tensors of the model's TTNO on ``tree`` from the state diagram
    (shifted frame, real FP64).  Returns W (oracle.ttno layout)."""
    n = tree.n
    node_of_mode = {tree.mode[u]: u for u in range(n) if tree.mode[u] >= 0}
    sub = [set(tree.subtree(u)) for u in range(n)]
    # items: ops = {mode: key} still carried as operators, coef, merged_at
    # (node whose parent edge merged it, or None), chan = {child node: channel}
    items = [{"ops": dict(t[1]), "coef": float(t[0]), "merged_at": None, "chan": {}} for t in model_terms(model)]
    nbond: Dict[int, int] = {}
    W: List[Optional[np.ndarray]] = [None] * n

    def local_key(it, u):
        m = tree.mode[u]
        return it["ops"].get(m) if m >= 0 else None

    def local_op(key, u):
        d = tree.phys[u]
        return np.eye(d) if key is None else _op_matrix(model, tree.mode[u], key, basis)

    for u in _post_order(tree):
        ch = tree.children(u)
        d = tree.phys[u]
        desc = [(local_key(it, u), tuple(it["chan"][c] for c in ch)) for it in items]
        if tree.parent[u] < 0:
            Wu = np.zeros(tuple(nbond[c] for c in ch) + (d, d))
            for it, (key, chs) in zip(items, desc):
                Wu[chs] += it["coef"] * local_op(key, u)
            W[u] = Wu
            break
        rights = [tuple(sorted((m, k) for m, k in it["ops"].items() if node_of_mode[m] not in sub[u])) for it in items]
        lid: Dict = {}
        rid: Dict = {}
        for dsc, r in zip(desc, rights):
            lid.setdefault(dsc, len(lid))
            rid.setdefault(r, len(rid))
        adj: List[List[int]] = [[] for _ in range(len(lid))]
        for dsc, r in zip(desc, rights):
            if rid[r] not in adj[lid[dsc]]:
                adj[lid[dsc]].append(rid[r])
        forced = sorted({lid[dsc] for it, dsc in zip(items, desc)
                         if it["merged_at"] is not None and it["merged_at"] not in sub[u]})
        cl, cr = min_vertex_cover(len(lid), len(rid), adj, forced)
        cl_set, cr_set = set(cl), set(cr)
        chan_l = {l: i for i, l in enumerate(cl)}
        chan_r = {r: len(cl) + i for i, r in enumerate(cr)}
        M = len(cl) + len(cr)
        nbond[u] = M
        Wu = np.zeros((M,) + tuple(nbond[c] for c in ch) + (d, d))
        inv_l = {v: k for k, v in lid.items()}
        for l in cl:  # descriptor channels, coefficient 1
            key, chs = inv_l[l]
            Wu[(chan_l[l],) + chs] += local_op(key, u)
        new_items = []
        merged: Dict[int, dict] = {}
        for it, dsc, r in zip(items, desc, rights):
            l, rr = lid[dsc], rid[r]
            if l in cl_set:
                it = dict(it)
                it["chan"] = dict(it["chan"])
                it["chan"][u] = chan_l[l]
                new_items.append(it)
                continue
            assert rr in cr_set, "vertex cover misses an item"
            key, chs = dsc
            Wu[(chan_r[rr],) + chs] += it["coef"] * local_op(key, u)
            if rr not in merged:
                # the channels of edges outside subtree(u) seen so far are the
                # members' (their operators there coincide and none of them was
                # merged there: those are left-covered above)
                chan = {e: v for e, v in it["chan"].items() if e not in sub[u]}
                chan[u] = chan_r[rr]
                merged[rr] = {"ops": {m: k for m, k in it["ops"].items() if node_of_mode[m] not in sub[u]},
                              "coef": 1.0, "merged_at": u, "chan": chan}
                new_items.append(merged[rr])
        items = new_items
        W[u] = Wu
    return W
