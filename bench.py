#!/usr/bin/env python3
"""Throughput benchmark of the TTNO x TTNS-block hot path on one MI355X.

Workload (default): the 64-mode coupled-oscillator Hamiltonian (all-pairs
quadratic couplings + 200 cubic terms, 8 harmonic-oscillator functions per
mode) on the balanced binary tree with physical legs on its 64 leaves (127
nodes), bond dimension 24, a block of k = 50 states.  The TTNO is compiled by
the library's own host compiler; the initial block is the seeded lowest
harmonic product states padded with noise.

One step = one block-LOBPCG outer iteration on the GPU: Rayleigh quotients,
residual fitting, the ALS preconditioner (2 sweeps, MINRES <= 10 per local
solve), Gram matrices over the 3k-state subspace, Rayleigh-Ritz and the
fitted recombination.  value = algorithmic contraction GFLOP/s over the timed
steps (minimum-flop orders, dense operands, per-state environments; every
contraction the step launches counts, nothing else does).

Also reported: time-to-all-states on the 6-mode workload (the configuration
with an exact reference) for the plain FP64 path and the mixed path, the
dominant kernel's roofline fraction, and the FP64 oracle timed on the host.
Prints one JSON line.
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


def make_solver(api, ctx, workload: str, precision: str, k: int, D: int):
    import workloads as wl
    from paper_2512_15875_amd.solver import TTNEigensolver

    if workload == "c2":
        model = wl.make_config_model("c2")
        tree = wl.binary_tree(model.dims)
    elif workload == "c3":
        model = wl.make_config_model("c3")
        tree = wl.fork_tree(model.dims, 4, 1)
    else:
        model = wl.make_config_model("c1")
        tree = wl.mps_tree(model.dims, 2)
    bonds = wl.bond_dims(tree, D)
    x0 = wl.initial_block(tree, bonds, model.omega, model.dims, k, model.seed + 17)
    s = TTNEigensolver(ctx, tree, model, D=D, k=k, precision=precision)
    s.load_block(x0)
    return s, model, tree


def time_to_all_states(api, ctx, precision: str, tol: float = 1e-3, max_iter: int = 12):
    """Solver start (block on the device) to the first LOBPCG iteration whose
    Rayleigh quotients all lie within tol of the exact levels (6-mode
    workload, MPS, D=8, k=10)."""
    import torch
    from paper_2512_15875_amd.solver import LobpcgOpts

    # exact normal-mode levels stored with the oracle runs (tests/golden/make_golden.py)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "c1_oracle_runs.json")))
    s, model, tree = make_solver(api, ctx, "c1", precision, 10, 8)
    ref = np.array(gold["exact"]) + gold["zpe"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.lobpcg_start(LobpcgOpts(n_iter=max_iter))
    hit = None
    for it in range(max_iter):
        s.lobpcg_step()
        lam = np.sort(s.lam_d.cpu().numpy() + s.zpe)
        if np.max(np.abs(lam - ref)) <= tol:
            hit = (it + 1, time.perf_counter() - t0, float(np.max(np.abs(lam - ref))))
            break
    return hit


def cpu_baseline(s, k: int, budget_s: float = 12.0):
    """The FP64 oracle's H_eff apply at the heaviest node, timed on the host."""
    from oracle import ttn as ottn

    tree = s.wtree
    u = tree.children(tree.root)[0]
    nb = tree.neighbours(u)
    rng = np.random.default_rng(7)
    edge = lambda c: u if c == tree.parent[u] else c
    W = rng.normal(size=tuple(s.M[edge(c)] for c in nb) + (1, 1))
    Db = [s.bonds[edge(c)] for c in nb]
    t0 = time.perf_counter()
    n = 0
    while True:
        X = rng.normal(size=tuple(Db) + (1,))
        E = {c: rng.normal(size=(Db[i], s.M[edge(c)], Db[i])) for i, c in enumerate(nb)}
        ottn.heff_apply(tree, u, W, X, E)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= k:
            break
    return u, n, time.perf_counter() - t0


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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16"])
    ap.add_argument("--workload", default="c2", choices=["c2", "c3"])
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--bond", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path (DESIGN.md describes how the "
              "hot path would shard)", file=sys.stderr)
        sys.exit(2)
    k = args.k or (50 if args.workload == "c2" else 84)
    D = args.bond or (24 if args.workload == "c2" else 40)

    import torch
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import LobpcgOpts

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    ctx = api.Context(0, workspace_bytes=8 << 30)
    s, model, tree = make_solver(api, ctx, args.workload, args.precision, k, D)
    s.lobpcg_start(LobpcgOpts(n_iter=args.warmup + args.steps + 1))
    print(f"setup done: {tree.n} nodes, k={k}, D={D}, precision={args.precision}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        s.lobpcg_step()
        print(f"warmup step {i} done", file=sys.stderr, flush=True)
    ctx.sync()
    torch.cuda.synchronize()
    api.ctx_flops(ctx, reset=True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        s.lobpcg_step()
        print(f"step {i} done: lam0={s.history[-1]['lam'].min():.4f} max|r|={s.history[-1]['resid'].max():.3e}",
              file=sys.stderr, flush=True)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flops = api.ctx_flops(ctx)
    ms = (t1 - t0) * 1e3 / args.steps
    value = flops / (t1 - t0) / 1e9

    # dominant contraction stage of one more step, timed with HIP events on the library stream
    api.profile(ctx, True)
    s.lobpcg_step()
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    by_kernel = {}
    for key, st, kern, cnt, tms, fl, *_ in rep:
        a = by_kernel.setdefault(kern, [0, 0.0, 0.0])
        a[0] += cnt
        a[1] += tms
        a[2] += fl
    for r in sorted(rep, key=lambda r: -r[4])[:12]:
        key, st, kern, cnt, tms, fl, Mm, Nn, Kk, nz = r
        print(f"  stage {key}#{st} {kern} M={Mm} N={Nn} K={Kk} items={nz} launches={cnt}: {tms:.1f} ms, "
              f"{fl / tms / 1e9:.1f} TFLOP/s", file=sys.stderr)
    by_class = {}
    for key, st, kern, cnt, tms, fl, Mm, Nn, Kk, nz in rep:
        cls = key.split(":")[0] + (":H" if key.split(":")[2] == "1" else ":I") + f":{kern.split('<')[1].split(',')[1].strip()}x{kern.split(',')[2].strip()}"
        a = by_class.setdefault(cls, [0, 0.0, 0.0])
        a[0] += cnt
        a[1] += tms
        a[2] += fl
    for cls, (cnt, tms, fl) in sorted(by_class.items(), key=lambda kv: -kv[1][1])[:10]:
        print(f"  class {cls}: {cnt} launches {tms:.1f} ms {fl / tms / 1e9:.1f} TFLOP/s", file=sys.stderr)
    dkern, (dcnt, dms, dfl) = max(by_kernel.items(), key=lambda kv: kv[1][1])
    achieved = dfl / (dms * 1e-3) / 1e12
    tot_ms = sum(v[1] for v in by_kernel.values())
    print(f"dominant kernel {dkern}: {dcnt} launches, {dms:.1f} ms total ({dms / dcnt:.4f} ms avg), "
          f"{achieved:.2f} TFLOP/s; all contraction stages {tot_ms:.1f} ms", file=sys.stderr, flush=True)

    workload_name = ("64-mode coupled oscillators + 200 cubic terms, binary leaf-only tree (127 nodes)"
                     if args.workload == "c2" else
                     "12-mode synthetic quartic force field (108 cubic + 191 quartic), fork-4 comb (16 nodes)")
    out = {
        "metric": "H_eff block-apply GFLOP/s (% MFMA peak); time-to-all-states at 1e-3 cm^-1 vs plain",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{workload_name}, D={D}, k={k}: one block-LOBPCG iteration (residual fit, ALS "
                               f"preconditioner 2 sweeps x MINRES<=10, 3k-subspace Gram + Rayleigh-Ritz, fitted "
                               f"recombination)",
                   "precision": args.precision, "gflop_per_step": round(flops / args.steps / 1e9, 2)},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK[args.precision],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK[args.precision], 4), "traffic": None,
                     "kernel": dkern, "launches": dcnt, "avg_ms": round(dms / dcnt, 5)},
    }
    if not args.no_tts:
        tts = {}
        for prec in ("fp64", "fp32"):
            c2 = api.Context(0, workspace_bytes=1 << 30)
            hit = time_to_all_states(api, c2, prec)
            tts[prec] = None if hit is None else {"iters": hit[0], "seconds": round(hit[1], 3),
                                                  "max_err_cm-1": hit[2]}
            c2.close()
        out["time_to_all_states"] = {"workload": "6-mode coupled oscillators, MPS, D=8, k=10 (exact reference)",
                                     "tol_cm-1": 1e-3, **tts}
    if not args.no_cpu_baseline:
        u, n, dt = cpu_baseline(s, k)
        # flops of one state's H_eff apply at node u (library count)
        envs = api.Envs(ctx, s.gt, 1, s.bonds, s.M, s.bonds, s.sdt,
                        edges=[api.dslot(s.gt, c, u) for c in s.gt.nbrs(u)])
        f1 = api.flops_heff(s.gt, s.op, envs, u, 1)
        out["cpu_baseline"] = {"value": round(f1 * n / dt / 1e9, 3), "unit": "GFLOP/s", "cores": blas_threads(),
                               "kind": "oracle",
                               "sample": f"FP64 NumPy H_eff apply at the level-1 node (n_loc="
                                         f"{int(np.prod(s.B.legdims(u)))}), {n} states in {dt:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
