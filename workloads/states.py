"""Seeded initial blocks and random tensors (inputs only).

Initial block: the k lowest harmonic product states |n_1 ... n_L>, ordered by
sum_i omega_i n_i (ties broken by the lexicographically smaller occupation
vector).  Each is a bond-1 tree tensor network state (one-hot tensors) embedded
at index 0 of every bond of dimension D_e, plus N(0, noise^2) entries drawn
with ``default_rng(seed)`` in the order state -> node -> row-major entry.
The tensors are returned un-normalised and un-gauged: each consumer brings the
block to canonical form with its own QR.
"""
from __future__ import annotations

import heapq
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .trees import Tree


def node_shape(tree: Tree, bonds: Sequence[int], u: int) -> Tuple[int, ...]:
    """Leg dims of node u in the order [parent, children..., physical]."""
    legs = []
    if tree.parent[u] >= 0:
        legs.append(bonds[u])
    for c in tree.children(u):
        legs.append(bonds[c])
    legs.append(tree.phys[u])
    return tuple(int(x) for x in legs)


def lowest_product_states(omega: Sequence[float], dims: Sequence[int], k: int) -> List[Tuple[int, ...]]:
    """The k occupation vectors of lowest sum_i omega_i n_i with 0 <= n_i < d_i
    (best-first enumeration; ties by lexicographic order of the vector)."""
    L = len(omega)
    start = tuple([0] * L)
    heap = [(0.0, start)]
    seen = {start}
    out: List[Tuple[int, ...]] = []
    while heap and len(out) < k:
        e, n = heapq.heappop(heap)
        out.append(n)
        for i in range(L):
            if n[i] + 1 < dims[i]:
                m = list(n)
                m[i] += 1
                m = tuple(m)
                if m not in seen:
                    seen.add(m)
                    heapq.heappush(heap, (e + float(omega[i]), m))
    # the heap pops equal energies in lexicographic order of the tuple
    return out


def initial_block(tree: Tree, bonds: Sequence[int], omega, dims, k: int, seed: int,
                  noise: float = 1e-2) -> List[List[np.ndarray]]:
    """[state][node] float64 tensors of the initial block (see module doc)."""
    occ = lowest_product_states(omega, dims, k)
    rng = np.random.default_rng(seed)
    block = []
    for j in range(k):
        tens = []
        for u in range(tree.n):
            shp = node_shape(tree, bonds, u)
            t = rng.normal(0.0, noise, size=shp)
            idx = [0] * (len(shp) - 1)
            p = occ[j][tree.mode[u]] if tree.mode[u] >= 0 else 0
            t[tuple(idx + [p])] += 1.0
            tens.append(t)
        block.append(tens)
    return block


def random_tensor(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    return rng.normal(0.0, scale, size=tuple(shape))


def random_block(tree: Tree, bonds: Sequence[int], k: int, seed: int) -> List[List[np.ndarray]]:
    """k dense random states (N(0,1) entries) with the tree's shapes."""
    rng = np.random.default_rng(seed)
    return [[rng.normal(0.0, 1.0, size=node_shape(tree, bonds, u)) for u in range(tree.n)] for _ in range(k)]


def sketch_matrices(tree: Tree, n: int, seed: int) -> List[Optional[np.ndarray]]:
    """Gaussian test matrices of a Khatri-Rao sketch: [d_u x n] N(0, 1) at
    every physical node (None at auxiliary nodes), drawn node by node."""
    rng = np.random.default_rng(seed)
    return [rng.normal(0.0, 1.0, size=(tree.phys[u], n)) if tree.phys[u] > 1 else None for u in range(tree.n)]
