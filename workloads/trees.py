"""Tree topologies for the TTNS/TTNO (inputs only).

A tree is given by ``parent[u]`` (-1 at the root), ``phys[u]`` (the physical
dimension; 1 for an auxiliary node) and ``mode[u]`` (the vibrational mode the
node carries, -1 for an auxiliary node).  Children of a node are ordered by
increasing node id; the leg order of every node tensor is
[parent, children..., physical] (Eq. ttns, Eq. ttno).

Topologies follow the paper (Appendix B): the linear MPS; the T tree (one
auxiliary node joining three chains of physical nodes); the balanced binary
tree with physical legs only on its leaves (leaf-only / ML-MCTDH-like) and the
paper's own 12-mode leaf-only tree; the fork-n (comb) trees: a chain of n
auxiliary backbone nodes, each carrying a chain of physical nodes; and the
12-mode full T3NS tree, where physical nodes and three-leg auxiliary nodes
alternate.
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


def _from_edges(name: str, n: int, root: int, edges, phys_of, mode_of) -> Tree:
    """Tree over nodes 0..n-1 from undirected edges, oriented away from root."""
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    parent = [-2] * n
    parent[root] = -1
    stack = [root]
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if parent[v] == -2:
                parent[v] = u
                stack.append(v)
    if any(p == -2 for p in parent):
        raise ValueError("edges do not connect the tree")
    return Tree(name, parent, [phys_of(u) for u in range(n)], [mode_of(u) for u in range(n)])


def t_tree(dims: List[int], arms: List[int]) -> Tree:
    """T tree: one auxiliary node (id 0, the root) joining three chains of
    physical nodes of lengths arms[0..2]; modes are assigned chain by chain
    from the first chain's far end inward (modes 1..arms[0] of the paper's
    figure run toward the junction), then outward along the second and third
    chains.  Node id 1 + m carries mode m."""
    L = len(dims)
    assert sum(arms) == L and len(arms) == 3
    edges = []
    a0, a1, a2 = arms
    # first chain: modes 0..a0-1, mode a0-1 next to the junction
    for m in range(a0 - 1):
        edges.append((1 + m, 2 + m))
    edges.append((1 + a0 - 1, 0))
    # second and third chains: from the junction outward
    start = a0
    for arm in (a1, a2):
        edges.append((0, 1 + start))
        for m in range(start, start + arm - 1):
            edges.append((1 + m, 2 + m))
        start += arm
    return _from_edges(f"ttree{L}", L + 1, 0, edges, lambda u: 1 if u == 0 else dims[u - 1],
                       lambda u: -1 if u == 0 else u - 1)


def leaf_only_12(dims: List[int]) -> Tree:
    """The paper's 12-mode leaf-only tree (Appendix B): auxiliary root with two
    auxiliary subtrees; modes at the leaves only.  Auxiliary ids 0..10
    (0 = root), mode m at node 11 + m; the branch pattern is the figure's
    (modes counted from 1 there): left ((5, 6), 1), ((7, 8), (9, 10)); right
    (11, 12), (3, (2, 4))."""
    assert len(dims) == 12
    leaf = lambda m: 11 + (m - 1)  # paper mode number -> node id
    # auxiliary: 0 root, 1 L10, 2 L21, 3 L42, 4 L11, 5 L22, 6 L12, 7 R10, 8 R21, 9 R11, 10 R12
    edges = [(0, 1), (1, 2), (2, 3), (3, leaf(5)), (3, leaf(6)), (2, leaf(1)),
             (1, 4), (4, 5), (5, leaf(7)), (5, leaf(8)), (4, 6), (6, leaf(9)), (6, leaf(10)),
             (0, 7), (7, 8), (8, leaf(11)), (8, leaf(12)), (7, 9), (9, leaf(3)), (9, 10), (10, leaf(2)),
             (10, leaf(4))]
    return _from_edges("leafonly12", 23, 0, edges, lambda u: 1 if u < 11 else dims[u - 11],
                       lambda u: -1 if u < 11 else u - 11)


def full_t3ns_12(dims: List[int]) -> Tree:
    """The paper's 12-mode full T3NS tree (Appendix B): physical node 1 (the
    root) joins auxiliary b1, b2; b1 joins physical 2 and 5, b2 joins 8 and
    11; each of 2, 5, 8, 11 carries an auxiliary node with the pairs (3, 4),
    (6, 7), (9, 10) and the single 12.  Mode m (1-based in the figure) sits at
    node m - 1; auxiliary nodes are 12..17 (b1..b6)."""
    assert len(dims) == 12
    c = lambda m: m - 1
    b = lambda i: 11 + i  # b1 -> 12 ... b6 -> 17
    edges = [(c(1), b(1)), (c(1), b(2)), (b(1), c(2)), (b(1), c(5)), (b(2), c(8)), (b(2), c(11)),
             (c(2), b(3)), (c(5), b(4)), (c(8), b(5)), (c(11), b(6)),
             (b(3), c(3)), (b(3), c(4)), (b(4), c(6)), (b(4), c(7)), (b(5), c(9)), (b(5), c(10)), (b(6), c(12))]
    return _from_edges("t3ns12", 18, 0, edges, lambda u: dims[u] if u < 12 else 1, lambda u: u if u < 12 else -1)


def paper_topology(name: str, dims: List[int]) -> Tree:
    """The topologies of the paper's 12-mode comparison (Table tab:ch3cn_summary):
    mps, ttree, leafonly, fork3, fork4, fork6, t3ns.  MPS is rooted at its
    middle site, the forks at their second backbone node, the T tree at its
    junction, the leaf-only and T3NS trees as drawn."""
    L = len(dims)
    if name == "mps":
        return mps_tree(dims, L // 2 - 1)
    if name == "ttree":
        a = -(-L // 3)
        return t_tree(dims, [a, a, L - 2 * a])
    if name == "leafonly":
        return leaf_only_12(dims) if L == 12 else binary_tree(dims)
    if name in ("fork3", "fork4", "fork6"):
        return fork_tree(dims, int(name[4:]), 1)
    if name == "t3ns":
        return full_t3ns_12(dims)
    raise ValueError(name)


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
