#!/usr/bin/env python3
"""Throughput benchmark of the TTNO x TTNS-block hot path on one MI355X.

Workload: the 64-mode coupled-oscillator Hamiltonian (all-pairs quadratic
couplings + 200 cubic terms, 8 harmonic-oscillator functions per mode) on the
balanced binary tree with physical legs on its 64 leaves (127 nodes), bond
dimension 24, a block of k = 50 states.  The TTNO is compiled by the library's
own host compiler; the block is seeded random data of the block's shapes.

One step = the contraction work of one ALS sweep over the tree for the whole
block: every directed-edge environment update (k pairs each; both directions
of all 126 edges, in dependency order) and the block H_eff product at all 127
nodes.  value = algorithmic contraction GFLOP/s over the timed steps
(minimum-flop contraction orders, dense operands, per-state environments).

Prints one JSON line (see the bench contract in the design doc).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0}  # dense MFMA TFLOP/s (vendor)


def build_workload(api, ctx, prec: str, k: int, D: int, seed: int = 2):
    import torch
    import workloads as wl

    model = wl.make_config_model("c2")
    tree = wl.binary_tree(model.dims)
    gt = api.Tree(tree.parent, tree.phys)
    W, M = api.sop_build(gt, tree.mode, model.omega, model.dims, model.monomials, model.coefs)
    sdt = api.F64 if prec == "fp64" else api.F32
    tdt = torch.float64 if sdt == api.F64 else torch.float32
    Wd = [torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=tdt) for w in W]
    op = api.TTNO(ctx, gt, Wd, [max(1, m) for m in M], sdt)
    bonds = wl.bond_dims(tree, D)
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], sdt)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    for u in range(tree.n):
        blk.t[u].normal_(generator=g)
    envs = api.Envs(ctx, gt, k, [max(1, b) for b in bonds], [max(1, m) for m in M], [max(1, b) for b in bonds], sdt)
    pairs = torch.arange(k, dtype=torch.int32, device="cuda")
    n_loc_max = max(int(np.prod(blk.legdims(u))) for u in range(tree.n))
    Y = torch.empty((k, n_loc_max), dtype=tdt, device="cuda")
    return dict(model=model, tree=tree, gt=gt, op=op, blk=blk, envs=envs, pairs=pairs, Y=Y, M=M, bonds=bonds,
                W=Wd)


def edge_order(tree):
    """Directed edges in dependency order: all u->parent in post-order, then
    all parent->u in pre-order."""
    post, pre = [], []

    def rec(u):
        pre.append(u)
        for c in tree.children(u):
            rec(c)
        post.append(u)

    rec(tree.root)
    up = [(u, tree.parent[u]) for u in post if tree.parent[u] >= 0]
    down = [(tree.parent[u], u) for u in pre if tree.parent[u] >= 0]
    return up + down


def make_step(api, ctx, w, compute, k):
    tree, gt, op, blk, envs, pairs, Y = w["tree"], w["gt"], w["op"], w["blk"], w["envs"], w["pairs"], w["Y"]
    edges = edge_order(tree)

    def step():
        for (u, v) in edges:
            api.ttno_env_update(ctx, gt, op, blk, blk, pairs, pairs, u, v, envs, compute)
        for u in range(tree.n):
            api.heff_apply_block(ctx, gt, op, envs, u, k, blk.t[u].view(k, -1), Y, flags=api.HEFF_NO_SHIFT,
                                 compute=compute)

    flops = 0.0
    for (u, v) in edges:
        flops += api.flops_env(gt, op, blk, blk, u, v) * k
    for u in range(tree.n):
        flops += api.flops_heff(gt, op, envs, u, k)
    return step, flops


def cpu_baseline(w, k, budget_s: float = 12.0):
    """The FP64 oracle's H_eff apply at the heaviest node, timed on the host."""
    from oracle import ttn as ottn

    tree, M, bonds = w["tree"], w["M"], w["bonds"]
    blk = w["blk"]
    # heaviest node by heff flops: the level-1 auxiliary node (child of the root)
    u = tree.children(tree.root)[0]
    nb = tree.neighbours(u)
    rng = np.random.default_rng(7)
    edge = lambda c: u if c == tree.parent[u] else c
    W = rng.normal(size=tuple(M[edge(c)] for c in nb) + (1, 1))
    Db = [bonds[edge(c)] for c in nb]
    flops_per_state = None
    t0 = time.perf_counter()
    n = 0
    while True:
        X = rng.normal(size=tuple(Db) + (1,))
        E = {c: rng.normal(size=(Db[i], M[edge(c)], Db[i])) for i, c in enumerate(nb)}
        ottn.heff_apply(tree, u, W, X, E)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= k:
            break
    dt = time.perf_counter() - t0
    return u, n, dt


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:
        return 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--bond", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (see DESIGN.md for how the "
              "hot path would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_15875_amd import ttn as api

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    compute = {"fp32": api.F32, "fp64": api.F64, "bf16": api.BF16}[args.precision]
    ctx = api.Context(0, workspace_bytes=8 << 30)
    w = build_workload(api, ctx, args.precision, args.k, args.bond)
    step, flops = make_step(api, ctx, w, compute, args.k)
    print(f"setup done: {w['tree'].n} nodes, k={args.k}, D={args.bond}, {flops / 1e9:.1f} GFLOP per step",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = flops * args.steps / (t1 - t0) / 1e9

    # dominant stage, timed with HIP events on the library stream
    api.profile(ctx, True)
    step()
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    by_kernel = {}
    for key, st, kern, cnt, tms, fl in rep:
        a = by_kernel.setdefault((key, st), [kern, 0, 0.0, 0.0])
        a[1] += cnt
        a[2] += tms
        a[3] += fl
    dom = max(by_kernel.items(), key=lambda kv: kv[1][2])
    (dkey, dst), (dkern, dcnt, dms, dfl) = dom
    achieved = dfl / (dms * 1e-3) / 1e12
    total_prof_ms = sum(v[2] for v in by_kernel.values())
    print(f"dominant stage {dkey} #{dst} {dkern}: {dcnt} launches, {dms / dcnt:.3f} ms avg, "
          f"{achieved:.1f} TFLOP/s; stages sum {total_prof_ms:.2f} ms of {ms:.2f} ms/step", file=sys.stderr)

    out = {
        "metric": "H_eff block-apply GFLOP/s (% MFMA peak); time-to-all-states at 1e-3 cm^-1 vs plain",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"64-mode coupled oscillators + 200 cubic terms, binary leaf-only tree (127 nodes), "
                               f"D={args.bond}, k={args.k}: one ALS-sweep contraction pass (all directed env "
                               f"updates + block H_eff at every node)",
                   "precision": args.precision, "gflop_per_step": round(flops / 1e9, 3)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK[args.precision],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK[args.precision], 4), "traffic": None,
                     "kernel": dkern, "stage": f"{dkey}#{dst}", "avg_ms": round(dms / dcnt, 4)},
    }
    if not args.no_cpu_baseline:
        u, n, dt = cpu_baseline(w, args.k)
        f1 = api.flops_heff(w["gt"], w["op"], w["envs"], u, 1)
        out["cpu_baseline"] = {"value": round(f1 * n / dt / 1e9, 3), "unit": "GFLOP/s", "cores": blas_threads(),
                               "kind": "oracle",
                               "sample": f"FP64 NumPy H_eff apply at the level-1 node (n_loc={int(np.prod(w['blk'].legdims(u)))}), "
                                         f"{n} states in {dt:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
