"""Tree topologies for the TTNS/TTNO (inputs only).

A tree is given by ``parent[u]`` (-1 at the root), ``phys[u]`` (the physical
dimension; 1 for an auxiliary node) and ``mode[u]`` (the vibrational mode the
node carries, -1 for an auxiliary node).  Children of a node are ordered by
increasing node id; the leg order of every node tensor is
[parent, children..., physical] (Eq. ttns, Eq. ttno).

Topologies follow the paper: the linear MPS, the balanced binary tree with
physical legs only on its leaves (leaf-only / ML-MCTDH-like), and the fork-n
(comb) tree of Appendix B, Fig. fork4: a chain of n auxiliary backbone nodes,
each carrying a chain of physical nodes.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


@dataclasses.dataclass
class Tree:
    name: str
    parent: List[int]
    phys: List[int]
    mode: List[int]

    @property
    def n(self) -> int:
        return len(self.parent)

    @property
    def root(self) -> int:
        return self.parent.index(-1)

    def children(self, u: int) -> List[int]:
        return [v for v in range(self.n) if self.parent[v] == u]

    def neighbours(self, u: int) -> List[int]:
        p = [self.parent[u]] if self.parent[u] >= 0 else []
        return p + self.children(u)

    def subtree(self, u: int) -> List[int]:
        out, stack = [], [u]
        while stack:
            x = stack.pop()
            out.append(x)
            stack.extend(self.children(x))
        return sorted(out)

    def to_json(self) -> dict:
        return {"name": self.name, "parent": list(self.parent), "phys": list(self.phys), "mode": list(self.mode)}


def mps_tree(dims: List[int], root: int) -> Tree:
    """Linear chain over modes 0..L-1 (node id = mode), rooted at ``root``."""
    L = len(dims)
    parent = [i + 1 if i < root else (i - 1 if i > root else -1) for i in range(L)]
    return Tree(f"mps{L}", parent, list(dims), list(range(L)))


def binary_tree(dims: List[int]) -> Tree:
    """Balanced binary tree whose leaves carry modes 0..L-1 left to right and
    whose internal nodes are auxiliary; a subtree over n modes splits them
    ceil(n/2) | floor(n/2).  Node ids are assigned in preorder (root = 0)."""
    parent: List[int] = []
    phys: List[int] = []
    mode: List[int] = []

    def build(modes, par):
        uid = len(parent)
        parent.append(par)
        if len(modes) == 1:
            phys.append(dims[modes[0]])
            mode.append(modes[0])
            return
        phys.append(1)
        mode.append(-1)
        h = (len(modes) + 1) // 2
        build(modes[:h], uid)
        build(modes[h:], uid)

    build(list(range(len(dims))), -1)
    return Tree(f"binary{len(dims)}", parent, phys, mode)


def fork_tree(dims: List[int], n_backbone: int, root_backbone: int = 1) -> Tree:
    """Fork-n comb: backbone b_0..b_{n-1} (auxiliary chain), backbone node b_i
    carries a chain of physical nodes.  Modes are assigned in order: the first
    chain gets modes 0..c-1 from the backbone outward, and so on; chain
    lengths are ceil/floor of L/n.  Rooted at backbone node ``root_backbone``.
    Node ids: backbone 0..n-1, then chain nodes in mode order."""
    L = len(dims)
    base, extra = divmod(L, n_backbone)
    lens = [base + (1 if i < extra else 0) for i in range(n_backbone)]
    parent = [0] * n_backbone
    for i in range(n_backbone):
        if i < root_backbone:
            parent[i] = i + 1
        elif i > root_backbone:
            parent[i] = i - 1
        else:
            parent[i] = -1
    phys = [1] * n_backbone
    mode = [-1] * n_backbone
    m = 0
    for i in range(n_backbone):
        prev = i
        for _ in range(lens[i]):
            parent.append(prev)
            phys.append(dims[m])
            mode.append(m)
            prev = len(parent) - 1
            m += 1
    return Tree(f"fork{n_backbone}_L{L}", parent, phys, mode)


def bond_dims(tree: Tree, D: int) -> List[int]:
    """Bond dimension of the edge (u, parent(u)) for every non-root u (entry
    at the root is 0): min(D, product of physical dims on either side)."""
    logs = np.log(np.asarray(tree.phys, dtype=np.float64))
    total = float(np.sum(logs))
    out = []
    for u in range(tree.n):
        if tree.parent[u] < 0:
            out.append(0)
            continue
        inside = float(np.sum(logs[tree.subtree(u)]))
        side = min(inside, total - inside)
        cap = D if side > np.log(D) + 1e-9 else int(round(np.exp(side)))
        out.append(int(min(D, cap)))
    return out
