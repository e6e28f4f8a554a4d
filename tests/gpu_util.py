"""Helpers for the GPU tests: random node networks shared by the HIP call and
the oracle (identical inputs), built from the seeded workload generators."""
import numpy as np
import torch

import workloads as wl


def star_tree(kappa: int, d: int):
    """Node 1 with a parent (node 0) and kappa-1 children (nodes 2..kappa)."""
    parent = [-1, 0] + [1] * (kappa - 1)
    phys = [2, d] + [2] * (kappa - 1)
    mode = [0, 1] + list(range(2, kappa + 1))
    return wl.Tree(f"star{kappa}", parent, phys, mode)


def node_case(kappa, d, Db, M, Da, k, seed, op=True, n_slots=None):
    """Random W, X and per-state incoming environments at node 1 of a star."""
    tree = star_tree(kappa, d)
    rng = np.random.default_rng(seed)
    nb = tree.neighbours(1)
    W = rng.normal(size=tuple(M) + (d, d)) if op else None
    X = rng.normal(size=(k,) + tuple(Da) + (d,))
    ns = n_slots or k
    E = {c: rng.normal(size=(ns, Db[i], M[i] if op else 1, Da[i])) for i, c in enumerate(nb)}
    return tree, W, X, E


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


TOL = {0: 1e-12, 1: 2e-5, 2: 3e-2, 3: 2e-5}  # F64, F32, BF16, F64 storage with F32 arithmetic (norm-wise relative)
