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
HBM_TBS = 8.0  # HBM3E TB/s (vendor)
MARKER_N = 12345  # doubles scaled before and after the profiled step (grid of 49 x 256 threads)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")
GEMM_SOURCE = os.path.join(ROOT, "paper_2512_15875_amd", "csrc", "gemm.hip")


def gemm_source_hash() -> str:
    import hashlib
    return hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """(measured HBM bytes, compulsory bytes) per launch of `kernel` from the
    committed counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated, on
    the Gram launches of this workload), or None when there is none for this
    kernel or the GEMM source changed since it was taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith("traffic|"):
            _, kern, h, meas, comp = line.rstrip("\n").split("|")
            rec[kern] = (h, float(meas), float(comp))
    if kernel not in rec or rec[kernel][0] != gemm_source_hash():
        return None
    return rec[kernel][1], rec[kernel][2]


def calibrate_copy():
    """A plain device copy of known size (for scaling FETCH_SIZE / WRITE_SIZE)."""
    import torch
    n = 64 << 20  # 64 Mi floats = 256 MiB each way
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))


def make_problem(workload: str, k: int, D: int):
    import workloads as wl

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
    return model, tree, x0


ENV_BUDGET = 16 << 30  # bytes of Gram environments kept at once (the pair chunk follows from it)


def make_solver(api, ctx, workload: str, precision: str, k: int, D: int):
    from paper_2512_15875_amd.solver import TTNEigensolver

    model, tree, x0 = make_problem(workload, k, D)
    s = TTNEigensolver(ctx, tree, model, D=D, k=k, precision=precision, env_budget_bytes=ENV_BUDGET)
    s.load_block(x0)
    return s, model, tree


def time_to_all_states(api, ctx, precision: str, tol: float = 1e-3, max_iter: int = 12, switch_tol: float = 1e-2):
    """Solver start (block on the device) to the first LOBPCG iteration whose
    Rayleigh quotients all lie within tol of the exact levels (6-mode
    workload, MPS, D=8, k=10).  precision "mixed": FP32 LOBPCG until the
    largest change of a Rayleigh quotient between iterations drops below
    switch_tol, then promotion to FP64 and FP64 LOBPCG."""
    import torch
    from paper_2512_15875_amd.solver import LobpcgOpts, MixedEigensolver

    # exact normal-mode levels stored with the oracle runs (tests/golden/make_golden.py)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "c1_oracle_runs.json")))
    ref = np.array(gold["exact"]) + gold["zpe"]
    opts = LobpcgOpts(n_iter=max_iter)
    if precision == "mixed":
        model, tree, x0 = make_problem("c1", 10, 8)
        ms = MixedEigensolver(ctx, tree, model, D=8, k=10, low="fp32")
        ms.load_block(x0)
        s = ms.lo
    else:
        s, model, tree = make_solver(api, ctx, "c1", precision, 10, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.lobpcg_start(opts)
    prev = None
    for it in range(max_iter):
        s.lobpcg_step()
        lam = np.sort(s.lam_d.cpu().numpy() + s.zpe)
        if np.max(np.abs(lam - ref)) <= tol:
            return it + 1, time.perf_counter() - t0, float(np.max(np.abs(lam - ref)))
        if precision == "mixed" and s is ms.lo and prev is not None and np.max(np.abs(lam - prev)) < switch_tol:
            ms.promote()
            s = ms.hi
        prev = lam
    return None


def learned_experiment(args):
    """The learned local preconditioner end to end: harvest (b, diag - s) -> y
    pairs from plain FP64 MINRES solves of the ALS preconditioner's systems
    on seeded force fields of the 12-mode generator (seeds 5000...), train the
    network on the GPU, then run block LOBPCG on the held-out 12-mode
    workload (seed 3) with the DIAG, LEARNED and MINRES local maps, and MINRES
    from DIAG- or learned-corrected starts, and report iterations and time
    against a longer FP64 MINRES-preconditioned run."""
    import torch
    from paper_2512_15875_amd import ttn as api

    ctx = api.Context(0, workspace_bytes=8 << 30)
    out = {"experiment": "learned local preconditioner", "train": {}, "test": {}}
    if args.learned_params:
        # parameters of an earlier training run (saved by this experiment)
        p = torch.from_numpy(np.load(args.learned_params)).to(device="cuda", dtype=torch.float32)
        out["train"] = {"params": os.path.basename(args.learned_params)}
    else:
        p = _learned_train(args, ctx, out)
    _learned_test(args, ctx, out, p)


def _learned_train(args, ctx, out):
    import torch
    import workloads as wl
    from paper_2512_15875_amd.learned import Trainer, TrainOpts
    from paper_2512_15875_amd.solver import LobpcgOpts, TTNEigensolver

    t0 = time.perf_counter()
    Xs, Ts = [], []
    for f in range(args.fields):
        seed = 5000 + f
        model = wl.make_config_model("c3", seed=seed)
        tree = wl.fork_tree(model.dims, 4, 1)
        bonds = wl.bond_dims(tree, args.train_bond)
        x0 = wl.initial_block(tree, bonds, model.omega, model.dims, args.train_k, seed + 17)
        s = TTNEigensolver(ctx, tree, model, D=args.train_bond, k=args.train_k, precision="fp64")
        s.load_block(x0)
        s.lobpcg_start(LobpcgOpts(n_iter=2))
        s.lobpcg_step()
        s.lobpcg_step()
        X, T = s.harvest(rows_per_node=-(-args.rows_per_field // tree.n), maxiter=args.harvest_maxiter,
                         rtol=1e-10, seed=seed)
        Xs.append(X)
        Ts.append(T)
        del s
        print(f"field {seed}: {X.shape[0]} pairs ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    t_h = time.perf_counter() - t0
    tr = Trainer(ctx, seed=0)
    t1 = time.perf_counter()
    hist = tr.fit(X, T, TrainOpts(epochs=args.epochs, batch=4096, lr=1e-3),
                  log=lambda r: print(f"  epoch {r['epoch']}: train {r['train_mse']:.4e} val {r['val_mse']:.4e} "
                                      f"(DIAG alone {r['val_mse_diag']:.4e})", file=sys.stderr, flush=True))
    ctx.sync()
    n_pairs = int(X.shape[0])
    del X, T, Xs, Ts
    out["train"] = {"fields": args.fields, "pairs": n_pairs, "bond": args.train_bond, "k": args.train_k,
                    "harvest_s": round(t_h, 1), "train_s": round(time.perf_counter() - t1, 1),
                    "final": hist[-1]}
    np.save(os.path.join(args.out_dir, "learned_params.npy"), tr.p.cpu().numpy())
    return tr.p


def _learned_test(args, ctx, out, params):
    """Held-out test: LOBPCG on the 12-mode workload (seed 3) with each local
    map of the preconditioner; errors against the last iterate of a longer
    plain FP64 MINRES run.  In FP64 the MINRES test run is the reference run's
    own first iterations (the same computation)."""
    import torch
    import workloads as wl
    from paper_2512_15875_amd.solver import LobpcgOpts, TTNEigensolver

    model = wl.make_config_model("c3")
    tree = wl.fork_tree(model.dims, 4, 1)
    k, D = args.k or 84, args.bond or 40
    bonds = wl.bond_dims(tree, D)
    x0 = wl.initial_block(tree, bonds, model.omega, model.dims, k, model.seed + 17)
    runs = {}
    maps = args.learned_maps.split(",")
    reuse = args.precision == "fp64" and "minres" in maps and args.test_iters <= args.ref_iters
    plan = [("reference_fp64_minres", "fp64", "minres", args.ref_iters)] + [
        (f"{pc}_{args.precision}", args.precision, pc, args.test_iters) for pc in maps
        if not (reuse and pc == "minres")]
    for name, prec, pc, iters in plan:
        s = TTNEigensolver(ctx, tree, model, D=D, k=k, precision=prec)
        s.load_block(x0)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        s.lobpcg_start(LobpcgOpts(n_iter=iters, precond=pc, mlp=params if "learned" in pc else None))
        lam_hist, t_hist = [], []
        for it in range(iters):
            s.lobpcg_step()
            lam_hist.append(np.sort(s.lam_d.cpu().numpy() + s.zpe))
            t_hist.append(time.perf_counter() - ts)
            print(f"  {name} iteration {it + 1}: {t_hist[-1]:.1f} s, lam[0]={lam_hist[-1][0]:.4f}", file=sys.stderr,
                  flush=True)
        runs[name] = (lam_hist, t_hist)
        print(f"{name}: {iters} iterations in {t_hist[-1]:.1f} s; lam[0]={lam_hist[-1][0]:.4f} "
              f"lam[-1]={lam_hist[-1][-1]:.4f}", file=sys.stderr, flush=True)
        del s
    ref = runs["reference_fp64_minres"][0][-1]
    if reuse:
        lh, th = runs["reference_fp64_minres"]
        runs["minres_fp64"] = (lh[:args.test_iters], th[:args.test_iters])
    for name, (lh, th) in runs.items():
        err = [float(np.max(np.abs(l - ref))) for l in lh]
        hit = next((i for i, e in enumerate(err) if e <= 1e-3), None)
        out["test"][name] = {"iters": len(lh), "seconds": round(th[-1], 2), "s_per_iter": round(th[-1] / len(lh), 3),
                             "max_err_per_iter": [round(e, 5) for e in err],
                             "states_within_1e-3_per_iter": [int(np.sum(np.abs(l - ref) <= 1e-3)) for l in lh],
                             "iters_to_1e-3": None if hit is None else hit + 1,
                             "seconds_to_1e-3": None if hit is None else round(th[hit], 2)}
    out["test"]["workload"] = f"12-mode quartic force field (seed 3), fork-4 comb, D={D}, k={k}"
    print(json.dumps(out), flush=True)


def ensemble_experiment(args):
    """Batched serving-style ensemble: independent seeded Hamiltonians (even
    seeds: coupled oscillators on binary trees, odd: quartic force fields on
    fork-4 combs), each run for a few FP32 LOBPCG iterations plus FP64
    refinement.  Concurrent (own stream per member, thread pool, graph-replayed
    sweeps, autotuned tiles) against one-at-a-time (one stream, eager, default
    tiles); both run twice and the second (warm) run is timed."""
    import torch
    import workloads as wl
    from paper_2512_15875_amd.ensemble import Ensemble, EnsembleOpts

    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import build_ttno

    members = wl.ensemble_members(args.members, D_range=(args.ens_dmin, args.ens_dmax),
                                  k_range=(args.ens_kmin, args.ens_kmax), L_range=(8, args.ens_lmax))
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for m in members:  # host TTNO compilation, once per member
        model = m["model"]
        tree = wl.binary_tree(model.dims) if m["kind"] == "c4-binary" else wl.fork_tree(model.dims, 4, 1)
        m["ttno"] = build_ttno(api.Tree(tree.parent, tree.phys), tree, model)
        log(f"TTNO of member {m['seed']} ({m['kind']}, L={m['L']}): {time.perf_counter() - t0:.1f} s")
    out = {"experiment": "ensemble", "members": len(members),
           "recipe": f"seeds 4000-{4000 + len(members) - 1}, L 8-{args.ens_lmax}, D {args.ens_dmin}-{args.ens_dmax}, "
                     f"k {args.ens_kmin}-{args.ens_kmax}, {args.ens_iters} FP32 LOBPCG iterations + 1 FP64"}
    res = {}
    modes = (("one_at_a_time", False, False), ("concurrent_untuned", True, False), ("concurrent", True, True))
    for name, conc, tune in modes:
        o = EnsembleOpts(low="fp32", iters_low=args.ens_iters, iters_fp64=1, concurrent=conc, threads=8,
                         graphs=conc, autotune=tune, workspace_bytes=512 << 20)
        t0 = time.perf_counter()
        ens = Ensemble(members, o, log=log)
        t_setup = time.perf_counter() - t0
        lam1, dt1, fl1 = ens.run()
        print(f"{name}: first run {dt1:.2f} s", file=sys.stderr, flush=True)
        lam2, dt2, fl2 = ens.run()
        print(f"{name}: second run {dt2:.2f} s ({fl2 / dt2 / 1e12:.2f} TFLOP/s)", file=sys.stderr, flush=True)
        res[name] = {"setup_s": round(t_setup, 2), "first_run_s": round(dt1, 3), "warm_run_s": round(dt2, 3),
                     "algorithmic_tflop": round(fl2 / 1e12, 3), "tflop_per_s": round(fl2 / dt2 / 1e12, 3)}
        res[name + "_lam"] = lam2
        ens.close()
        del ens
        torch.cuda.synchronize()
    dev = lambda x, y: max(float(np.max(np.abs(a - b))) for a, b in zip(res[x + "_lam"], res[y + "_lam"]))
    for name, _, _ in modes:
        out[name] = res[name]
    out["speedup"] = round(res["one_at_a_time"]["warm_run_s"] / res["concurrent"]["warm_run_s"], 3)
    out["speedup_untuned"] = round(res["one_at_a_time"]["warm_run_s"] / res["concurrent_untuned"]["warm_run_s"], 3)
    # streams and graphs do not change the arithmetic: bitwise-equal eigenvalues expected
    out["max_eigenvalue_difference_untuned_cm-1"] = dev("one_at_a_time", "concurrent_untuned")
    # tuned tiles change FP32 summation order (amplified by the unconverged early iterations)
    out["max_eigenvalue_difference_tuned_cm-1"] = dev("one_at_a_time", "concurrent")
    print(json.dumps(out), flush=True)


def tts_experiment(args):
    """Time to all states at 1e-3 cm^-1 on a large workload: plain FP64 block
    LOBPCG for ref_iters iterations (its last iterate is the reference), then
    the mixed form (FP32 iterations until the largest change of a Rayleigh
    quotient between iterations drops below switch_tol, promotion, FP64
    iterations) from the same initial block; both timed from solver start."""
    import torch
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import LobpcgOpts, MixedEigensolver, TTNEigensolver, build_ttno

    wl_name = args.workload
    k = args.k or (50 if wl_name == "c2" else 84)
    D = args.bond or (24 if wl_name == "c2" else 40)
    model, tree, x0 = make_problem(wl_name, k, D)
    ctx = api.Context(0, workspace_bytes=8 << 30)
    ttno = build_ttno(api.Tree(tree.parent, tree.phys), tree, model)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    # plain FP64
    s = TTNEigensolver(ctx, tree, model, D=D, k=k, precision="fp64", ttno=ttno)
    s.load_block(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.lobpcg_start(LobpcgOpts(n_iter=args.ref_iters))
    plain = []
    for it in range(args.ref_iters):
        s.lobpcg_step()
        plain.append((time.perf_counter() - t0, np.sort(s.lam_d.cpu().numpy() + s.zpe)))
        log(f"  plain fp64 iteration {it + 1}: {plain[-1][0]:.1f} s")
    del s
    ref = plain[-1][1]

    def first_hit(traj):
        for i, t in enumerate(traj):
            if np.max(np.abs(t[1] - ref)) <= 1e-3 and (len(t) < 3 or t[2] == "fp64"):
                return i + 1, round(t[0], 2)
        return None, None

    pi, pt = first_hit(plain)
    out = {"experiment": "time to all states", "workload": f"{wl_name}, D={D}, k={k}", "tol_cm-1": 1e-3,
           "reference": f"plain FP64 LOBPCG iterate {args.ref_iters}",
           "plain_fp64": {"iters": pi, "seconds": pt, "s_per_iter": round(plain[-1][0] / len(plain), 3),
                          "max_err_per_iter": [round(float(np.max(np.abs(t[1] - ref))), 5) for t in plain]}}
    # mixed, once per arithmetic of the FP64 phase's preconditioner sweeps
    for pre in args.tts_pre.split(","):
        hi_pre = {"f64": None, "f64_f32": api.F64_F32}[pre]
        ms = MixedEigensolver(ctx, tree, model, D=D, k=k, low=args.precision, ttno=ttno, hi_pre_compute=hi_pre)
        ms.load_block(x0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cur = ms.lo
        cur.lobpcg_start(LobpcgOpts(n_iter=args.ref_iters))
        mixed, prev, switched = [], None, None
        for it in range(args.ref_iters):
            cur.lobpcg_step()
            lam = np.sort(cur.lam_d.cpu().numpy() + cur.zpe)
            mixed.append((time.perf_counter() - t0, lam, "lo" if cur is ms.lo else "fp64"))
            log(f"  mixed ({pre} preconditioner) iteration {it + 1} ({mixed[-1][2]}): {mixed[-1][0]:.1f} s, "
                f"max err {np.max(np.abs(lam - ref)):.4f}")
            if np.max(np.abs(lam - ref)) <= 1e-3 and cur is ms.hi:
                break
            if cur is ms.lo and prev is not None and np.max(np.abs(lam - prev)) < args.switch_tol:
                ms.promote()
                cur = ms.hi
                switched = it + 1
            prev = lam
        del ms
        mi, mt = first_hit(mixed)
        key = "mixed" if pre == "f64" else f"mixed_pre_{pre}"
        out[key] = {"low": args.precision, "fp64_phase_preconditioner": pre, "switch_at_iter": switched, "iters": mi,
                    "seconds": mt, "max_err_per_iter": [round(float(np.max(np.abs(t[1] - ref))), 5) for t in mixed]}
        if pt and mt:
            out["speedup" if pre == "f64" else f"speedup_pre_{pre}"] = round(pt / mt, 3)
    print(json.dumps(out), flush=True)


def ii_experiment(args):
    """Inverse-iteration refinement on a large workload: the mixed LOBPCG
    (FP32 iterations, promotion, FP64 iterations) brings the block close,
    then block inverse iteration in FP64 runs from the same block twice --
    local MINRES in FP64, and FP64 iterative refinement around MINRES in FP32
    matrix-core arithmetic -- each followed by the final global
    Rayleigh-Ritz."""
    import torch
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import IIOpts, LobpcgOpts, MixedEigensolver, build_ttno

    wl_name = args.workload
    k = args.k or (50 if wl_name == "c2" else 84)
    D = args.bond or (24 if wl_name == "c2" else 40)
    model, tree, x0 = make_problem(wl_name, k, D)
    ctx = api.Context(0, workspace_bytes=8 << 30)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    ms = MixedEigensolver(ctx, tree, model, D=D, k=k, low="fp32",
                          ttno=build_ttno(api.Tree(tree.parent, tree.phys), tree, model))
    ms.load_block(x0)
    t0 = time.perf_counter()
    ms.lo.lobpcg_start(LobpcgOpts(n_iter=args.ii_lo + args.ii_hi))
    for i in range(args.ii_lo):
        ms.lo.lobpcg_step()
        log(f"  fp32 LOBPCG {i + 1}: {time.perf_counter() - t0:.1f} s")
    ms.promote()
    for i in range(args.ii_hi):
        ms.hi.lobpcg_step()
        log(f"  fp64 LOBPCG {i + 1}: {time.perf_counter() - t0:.1f} s")
    s = ms.hi
    lam0 = np.sort(s.lam_d.cpu().numpy() + s.zpe)
    snap = [s.B.t[u][:k].clone() for u in range(s.gt.n)]
    lam_snap = s.lam_d.clone()
    out = {"experiment": "inverse iteration", "workload": f"{wl_name}, D={D}, k={k}",
           "lobpcg": f"{args.ii_lo} FP32 + {args.ii_hi} FP64 iterations, {time.perf_counter() - t0:.1f} s"}
    res = {}
    for name, refine in (("fp64_minres", 0), ("refined_fp32_minres", 2)):
        for u in range(s.gt.n):
            s.B.t[u][:k].copy_(snap[u])
        s.lam_d.copy_(lam_snap)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        theta = s.inverse_iteration(IIOpts(n_iter=args.ii_iters, minres_maxiter=args.ii_maxiter, minres_rtol=1e-10,
                                           refine=refine),
                                    log=lambda r: log(f"  {name} II {r['iter'] + 1}: {time.perf_counter() - t1:.1f} s"))
        ctx.sync()
        dt = time.perf_counter() - t1
        res[name] = np.sort(theta)
        out[name] = {"seconds": round(dt, 2), "iters": args.ii_iters,
                     "reverted_states": [len(h.get("reverted", [])) for h in s.history[-args.ii_iters:]],
                     "sum_lambda_change_cm-1": round(float(np.sum(res[name] - lam0)), 5),
                     "max_lambda_drop_cm-1": round(float(np.max(lam0 - res[name])), 5),
                     "max_lambda_rise_cm-1": round(float(np.max(res[name] - lam0)), 5)}
        log(f"{name}: {dt:.1f} s")
    out["max_difference_fp64_vs_refined_cm-1"] = float(np.max(np.abs(res["fp64_minres"] - res["refined_fp32_minres"])))
    out["speedup_refined"] = round(out["fp64_minres"]["seconds"] / out["refined_fp32_minres"]["seconds"], 3)
    print(json.dumps(out), flush=True)


def ienv_probe(args):
    """The fused identity overlap environment alone, for counter passes: a
    three-leg node with 24-dimensional bonds and no physical leg (the c2
    internal nodes), 150 random FP32 states, 20 000 random (bra, ket) pairs,
    one environment update toward each leg, timed and printed per leg."""
    import torch
    import workloads as wl
    from paper_2512_15875_amd import ttn as api

    ctx = api.Context(0, workspace_bytes=2 << 30)
    n, reps, ks, Dn = args.probe_pairs, args.probe_reps, 150, 24
    tree = wl.Tree("star3", [-1, 0, 1, 1], [2, 1, 2, 2], [0, 1, 2, 3])  # node 1: parent 0, children 2, 3
    gt = api.Tree(tree.parent, tree.phys)
    nb = tree.neighbours(1)
    bb = [1] * tree.n
    for c in nb:
        bb[1 if c == 0 else c] = Dn
    bra = api.Block(ctx, gt, ks, bb, api.F32)
    g = torch.Generator(device="cpu")
    g.manual_seed(0)
    bra.t[1].copy_(torch.randn(bra.t[1].shape, generator=g))
    envs = api.Envs(ctx, gt, n, bb, None, bb, api.F32)
    for c in nb:
        envs.get(c, 1).copy_(torch.randn(envs.get(c, 1).shape, generator=g))
    pb = torch.randint(0, ks, (n,), generator=g, dtype=torch.int32).cuda()
    pk = torch.randint(0, ks, (n,), generator=g, dtype=torch.int32).cuda()
    for v in nb:
        api.ttno_env_update(ctx, gt, None, bra, bra, pb, pk, 1, v, envs, api.F32)
    ctx.sync()
    for v in nb:
        t0 = time.perf_counter()
        for _ in range(reps):
            api.ttno_env_update(ctx, gt, None, bra, bra, pb, pk, 1, v, envs, api.F32)
        ctx.sync()
        dt = (time.perf_counter() - t0) / reps
        print(f"toward {v}: {dt * 1e3:.3f} ms for {n} pairs = {dt / n * 1e9:.1f} ns/pair, "
              f"{2 * Dn ** 4 * 3 * n / dt / 1e12:.1f} TFLOP/s", flush=True)


def gram_probe(args):
    """The Gram step of one LOBPCG iteration alone (environment updates and
    closures over all pairs of the 3k basis) at the bench workload, bracketed
    by the same markers as the profiled step; prints the per-kernel
    algorithmic flops and bytes per launch (for the counter passes, which
    rocprofv3 cannot take over a whole step)."""
    import torch
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import LobpcgOpts

    k = args.k or 50
    D = args.bond or 24
    ctx = api.Context(0, workspace_bytes=8 << 30)
    s, model, tree = make_solver(api, ctx, "c2", args.precision, k, D)
    s.lobpcg_start(LobpcgOpts(n_iter=1))
    m = 3 * k
    ia = [a for a in range(m) for b in range(a, m)]
    ib = [b for a in range(m) for b in range(a, m)]
    s.gram(s.B, ia, ib)  # warm: plans and tables
    ctx.sync()
    mark = torch.zeros(MARKER_N, dtype=torch.float64, device="cuda")
    api.vec_scale(ctx, mark, 1.0, mark)
    api.profile(ctx, True)
    s.gram(s.B, ia, ib)
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    api.vec_scale(ctx, mark, 1.0, mark)
    ctx.sync()
    by = {}
    for key, st, kern, cnt, tms, fl, *_rest in rep:
        a = by.setdefault(kern, [0, 0.0, 0.0, 0.0])
        a[0] += cnt
        a[1] += tms
        a[2] += fl
        a[3] += _rest[-1]
    out = {kern: {"launches": c, "avg_ms": round(t / c, 5), "algorithmic_flop_per_launch": f / c,
                  "algorithmic_bytes_per_launch": b / c} for kern, (c, t, f, b) in by.items()}
    print(json.dumps({"gram_probe": f"c2, D={D}, k={k}, {len(ia)} pairs", "kernels": out}), flush=True)


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
    ap.add_argument("--calibrate-copy", action="store_true", help="only run the copy kernel used to scale counters")
    ap.add_argument("--workspace-gb", type=float, default=8.0,
                    help="library workspace of the bench step (stage intermediates; bounds the items per launch)")
    ap.add_argument("--gram-probe", action="store_true", help="only the Gram step, for counter passes")
    ap.add_argument("--ienv-probe", action="store_true",
                    help="only the fused identity overlap environment at a 24x24x24 node, for counter passes")
    ap.add_argument("--probe-pairs", type=int, default=20000)
    ap.add_argument("--probe-reps", type=int, default=5)
    ap.add_argument("--ii", action="store_true", help="run the inverse-iteration experiment instead")
    ap.add_argument("--ii-lo", type=int, default=10)
    ap.add_argument("--ii-hi", type=int, default=4)
    ap.add_argument("--ii-iters", type=int, default=2)
    ap.add_argument("--ii-maxiter", type=int, default=200)
    ap.add_argument("--learned", action="store_true", help="run the learned-preconditioner experiment instead")
    ap.add_argument("--fields", type=int, default=32)
    ap.add_argument("--train-bond", type=int, default=24)
    ap.add_argument("--train-k", type=int, default=12)
    ap.add_argument("--rows-per-field", type=int, default=3000)
    ap.add_argument("--harvest-maxiter", type=int, default=300)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--test-iters", type=int, default=12)
    ap.add_argument("--learned-maps", default="diag,learned,minres,minres+diag,minres+learned",
                    help="local maps of the held-out LOBPCG runs (comma-separated)")
    ap.add_argument("--learned-params", default="",
                    help="saved network parameters (.npy) to test instead of harvesting and training")
    ap.add_argument("--ref-iters", type=int, default=24)
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "out"),
                    help="where experiments write their side files (learned parameters, per-iteration data)")
    ap.add_argument("--ensemble", action="store_true", help="run the many-Hamiltonian ensemble experiment instead")
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--ens-dmin", type=int, default=12)
    ap.add_argument("--ens-dmax", type=int, default=24)
    ap.add_argument("--ens-kmin", type=int, default=10)
    ap.add_argument("--ens-kmax", type=int, default=32)
    ap.add_argument("--ens-iters", type=int, default=3)
    ap.add_argument("--ens-lmax", type=int, default=32)
    ap.add_argument("--tts", action="store_true", help="run the plain-vs-mixed time-to-all-states experiment")
    ap.add_argument("--autotune", action="store_true",
                    help="measured tile choice on each stage's first launch (default: the planner's heuristic, "
                         "deterministic, so that profiles of the same command agree)")
    ap.add_argument("--graphs", action="store_true", help="replay the sweeps as HIP graphs (own stream)")
    ap.add_argument("--switch-tol", type=float, default=0.05)
    ap.add_argument("--tts-pre", default="f64",
                    help="arithmetic of the mixed form's FP64-phase preconditioner sweeps: f64, f64_f32 "
                         "(FP32 matrix cores on the FP64 tensors), or both comma-separated")
    ap.add_argument("--gemm-hash", action="store_true", help="print the GEMM source hash and exit")
    args = ap.parse_args()
    if args.graphs and args.warmup < 2:
        args.warmup = 2  # first step runs eagerly, the second captures: keep both untimed
    if args.gemm_hash:
        print(gemm_source_hash())
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path, so --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gram_probe:
        gram_probe(args)
        return
    if args.ienv_probe:
        ienv_probe(args)
        return
    if args.ii:
        ii_experiment(args)
        return
    if args.tts:
        tts_experiment(args)
        return
    if args.ensemble:
        ensemble_experiment(args)
        return
    if args.learned:
        os.makedirs(args.out_dir, exist_ok=True)
        learned_experiment(args)
        return
    k = args.k or (50 if args.workload == "c2" else 84)
    D = args.bond or (24 if args.workload == "c2" else 40)

    import torch
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import LobpcgOpts

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.graphs:
        # graphs need a non-null stream: the whole run goes on one of its own
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            run_bench(args, api, k, D, stream)
    else:
        run_bench(args, api, k, D, None)


def run_bench(args, api, k, D, stream):
    import torch
    from paper_2512_15875_amd.solver import LobpcgOpts

    ctx = api.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)), stream=stream)
    api.autotune(ctx, args.autotune)
    s, model, tree = make_solver(api, ctx, args.workload, args.precision, k, D)
    s.graphs = args.graphs
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

    # per-kernel totals of one more step, timed with HIP events on the library stream;
    # the step is bracketed by two copies of MARKER_N doubles (a launch of a
    # distinct grid size) so that counter and trace summaries can select it
    mark = torch.zeros(MARKER_N, dtype=torch.float64, device="cuda")
    api.vec_scale(ctx, mark, 1.0, mark)
    api.profile(ctx, True)
    s.lobpcg_step()
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    api.vec_scale(ctx, mark, 1.0, mark)
    ctx.sync()
    by_kernel = {}
    for key, st, kern, cnt, tms, fl, Mm, Nn, Kk, nz, by in rep:
        a = by_kernel.setdefault(kern, [0, 0.0, 0.0, 0.0])
        a[0] += cnt
        a[1] += tms
        a[2] += fl
        a[3] += by
    for r in sorted(rep, key=lambda r: -r[4])[:12]:
        key, st, kern, cnt, tms, fl, Mm, Nn, Kk, nz, by = r
        print(f"  stage {key}#{st} {kern} M={Mm} N={Nn} K={Kk} items={nz} launches={cnt}: {tms:.1f} ms, "
              f"{fl / tms / 1e9:.1f} TFLOP/s, {by / tms / 1e6:.0f} GB/s", file=sys.stderr)
    for kern, (cnt, tms, fl, by) in sorted(by_kernel.items(), key=lambda kv: -kv[1][1])[:8]:
        print(f"  kernel {kern}: {cnt} launches {tms:.1f} ms {fl / tms / 1e9:.1f} TFLOP/s "
              f"{by / tms / 1e6:.0f} GB/s intensity {fl / max(by, 1):.1f} flop/B", file=sys.stderr)
    dkern, (dcnt, dms, dfl, dby) = max(by_kernel.items(), key=lambda kv: kv[1][1])
    tot_ms = sum(v[1] for v in by_kernel.values())
    # the H_eff block applies of the step (every heff_apply_block with the TTNO:
    # the ALS preconditioner's MINRES products), grouped per call shape
    heff = {}
    for key, st, kern, cnt, tms, fl, Mm, Nn, Kk, nz, by in rep:
        parts = key.split(":")
        if parts[0] == "heff" and parts[2] == "1":
            a = heff.setdefault(parts[1], [0.0, 0.0])
            a[0] += fl
            a[1] += tms
    heff_fl = sum(v[0] for v in heff.values())
    heff_ms = sum(v[1] for v in heff.values())
    heavy_u, (hfl, hms) = max(heff.items(), key=lambda kv: kv[1][0]) if heff else ("-", (0.0, 1.0))
    heff_line = {"tflop_per_s": round(heff_fl / (heff_ms * 1e-3) / 1e12, 2) if heff_ms else None,
                 "frac_of_peak": round(heff_fl / (heff_ms * 1e-3) / 1e12 / PEAK[args.precision], 4) if heff_ms else None,
                 "ms_in_step": round(heff_ms, 1), "share_of_contraction_time": round(heff_ms / tot_ms, 3),
                 "heaviest_node": {"node": heavy_u, "tflop_per_s": round(hfl / (hms * 1e-3) / 1e12, 2),
                                   "frac_of_peak": round(hfl / (hms * 1e-3) / 1e12 / PEAK[args.precision], 4)}}
    peak_tf = PEAK[args.precision]
    ridge = peak_tf * 1e12 / (HBM_TBS * 1e12)
    if dfl / max(dby, 1.0) >= ridge:
        roof = {"bound": "mfma", "achieved": round(dfl / (dms * 1e-3) / 1e12, 3), "peak": peak_tf,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(dby / (dms * 1e-3) / 1e9, 1), "peak": HBM_TBS * 1e3,
                "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    tr = measured_traffic(dkern)
    # the counters cover this kernel's Gram launches (rocprofv3 cannot count a
    # whole step here): their measured / compulsory ratio applied to this
    # step's compulsory bytes per launch
    roof["traffic"] = None if tr is None else round(tr[0] / tr[1] * dby / dcnt, 0)
    if tr is not None:
        roof["traffic_unit"] = "bytes per launch"
        roof["traffic_over_compulsory"] = round(tr[0] / tr[1], 3)
        roof["traffic_source"] = "profiles/gram_c2_fp32_hbm_counters.md (Gram launches of this kernel)"
    roof.update({"kernel": dkern, "launches": dcnt, "avg_ms": round(dms / dcnt, 5),
                 "algorithmic_flop_per_launch": dfl / dcnt, "algorithmic_bytes_per_launch": dby / dcnt,
                 "share_of_contraction_time": round(dms / tot_ms, 3)})
    print(f"dominant kernel {dkern}: {dcnt} launches, {dms:.1f} ms total ({dms / dcnt:.4f} ms avg); all "
          f"contraction stages {tot_ms:.1f} ms", file=sys.stderr, flush=True)

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
                   "precision": args.precision, "gflop_per_step": round(flops / args.steps / 1e9, 2),
                   "autotune": bool(args.autotune), "graphs": bool(args.graphs)},
        "roofline": roof,
        "heff_apply_block": heff_line,
    }
    if not args.no_tts:
        tts = {}
        for prec in ("fp64", "fp32", "mixed"):
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
