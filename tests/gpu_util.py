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


def heff_setup(api, ctx, kappa, d, Db, M, Da, k, seed, dt, op=True):
    tree, W, X, E = node_case(kappa, d, Db, M, Da, k, seed, op=op)
    f64 = dt in (api.F64, api.F64_F32)  # FP64 tensors (the F64_F32 compute type reads FP64 storage)
    tdt = torch.float64 if f64 else torch.float32
    sdt = api.F64 if f64 else api.F32
    gt = api.Tree(tree.parent, tree.phys)
    bond = [0] + [0] * tree.n
    bond = [0] * tree.n
    nb = tree.neighbours(1)
    for i, c in enumerate(nb):
        e = 1 if c == 0 else c
        bond[e] = Db[i]
    kb = list(bond)
    for i, c in enumerate(nb):
        kb[1 if c == 0 else c] = Da[i]
    opb = [0] * tree.n
    for i, c in enumerate(nb):
        opb[1 if c == 0 else c] = M[i]
    gW = None
    if op:
        Wd = [to_dev(np.zeros((1,)), tdt) for _ in range(tree.n)]
        Wd[1] = to_dev(W, tdt)
        gW = api.TTNO(ctx, gt, Wd, [max(1, x) for x in opb], sdt)
    edges = [api.dslot(gt, c, 1) for c in nb]
    envs = api.Envs(ctx, gt, k, [max(1, x) for x in bond], [max(1, x) for x in opb] if op else None,
                    [max(1, x) for x in kb], sdt, edges=edges)
    for c in nb:
        envs.get(c, 1).copy_(to_dev(E[c], tdt))
    return tree, W, X, E, gt, gW, envs, tdt


def env_setup(api, ctx, kappa, d, Db, M, Da, kb, kk, seed, dt, op=True, toward_leg=0):
    tree = star_tree(kappa, d)
    rng = np.random.default_rng(seed)
    nb = tree.neighbours(1)
    tdt = torch.float64 if dt == api.F64 else torch.float32
    sdt = api.F64 if dt == api.F64 else api.F32
    gt = api.Tree(tree.parent, tree.phys)
    edge = lambda c: 1 if c == 0 else c
    bb, ab, mb = [1] * tree.n, [1] * tree.n, [1] * tree.n
    for i, c in enumerate(nb):
        bb[edge(c)], ab[edge(c)], mb[edge(c)] = Db[i], Da[i], M[i] if op else 1
    bra = api.Block(ctx, gt, kb, bb, sdt)
    ket = api.Block(ctx, gt, kk, ab, sdt)
    A_b = rng.normal(size=(kb,) + tuple(Db) + (d,))
    A_k = rng.normal(size=(kk,) + tuple(Da) + (d,))
    bra.t[1].copy_(to_dev(A_b, tdt))
    ket.t[1].copy_(to_dev(A_k, tdt))
    W = rng.normal(size=tuple(M) + (d, d)) if op else None
    gW = None
    if op:
        Wd = [to_dev(np.zeros((1,)), tdt) for _ in range(tree.n)]
        Wd[1] = to_dev(W, tdt)
        gW = api.TTNO(ctx, gt, Wd, mb, sdt)
    pairs = [(i, j) for i in range(kb) for j in range(kk)]
    npairs = len(pairs)
    envs = api.Envs(ctx, gt, npairs, bb, mb if op else None, ab, sdt)
    E = {}
    for i, c in enumerate(nb):
        E[c] = rng.normal(size=(npairs, Db[i], M[i] if op else 1, Da[i]))
        envs.get(c, 1).copy_(to_dev(E[c], tdt))
    pb = torch.tensor([p[0] for p in pairs], dtype=torch.int32, device="cuda")
    pk = torch.tensor([p[1] for p in pairs], dtype=torch.int32, device="cuda")
    return tree, gt, bra, ket, A_b, A_k, W, gW, envs, E, pairs, pb, pk, tdt


TOL = {0: 1e-12, 1: 1e-5, 2: 3e-2, 3: 1e-5}  # F64, F32, BF16, F64 storage with F32 arithmetic (norm-wise relative)
