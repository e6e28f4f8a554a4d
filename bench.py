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

PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16": 2500.0, "f64_f32": 157.3}  # dense MFMA TFLOP/s (vendor)
# (f64_f32: FP64 storage, the contractions on FP32 matrix cores)
HBM_TBS = 8.0  # HBM3E TB/s (vendor)
MARKER_N = 12345  # doubles scaled before and after the profiled step (grid of 49 x 256 threads)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.txt")
GEMM_SOURCE = os.path.join(ROOT, "paper_2512_15875_amd", "csrc", "gemm.hip")


def gemm_source_hash() -> str:
    import hashlib
    return hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str):
    """(measured HBM bytes, stage bytes) per launch of `kernel` from the
    committed counter summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated, on
    the launches of the headline U1 probe), or None when there is none for
    this kernel or the GEMM source changed since it was taken."""
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


def measured_u1_call_traffic():
    """(measured HBM bytes, compulsory U1 bytes) of one whole headline U1
    call (all its stages) from the same summary, or None (absent, or the
    GEMM source changed)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    for line in open(TRAFFIC_FILE):
        if line.startswith("u1call|"):
            _, h, meas, comp = line.rstrip("\n").split("|")
            if h == gemm_source_hash():
                return float(meas), float(comp)
    return None


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


def time_to_all_states(api, ctx, form: str, tol: float = 1e-3, max_iter: int = 12, switch_tol: float = 1e-2):
    """Solver start (block on the device) to the first LOBPCG iteration whose
    Rayleigh quotients all lie within tol of the exact levels (6-mode
    workload, MPS, D=8, k=10).  form: "fp64" (plain), "fp32", "f64_f32", or
    "mixed" (FP32-storage LOBPCG until the largest change of a Rayleigh
    quotient between iterations drops below switch_tol, then promotion and
    f64_f32 LOBPCG)."""
    import torch
    from paper_2512_15875_amd.solver import LobpcgOpts, MixedEigensolver

    # exact normal-mode levels stored with the oracle runs (tests/golden/make_golden.py)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "c1_oracle_runs.json")))
    ref = np.array(gold["exact"]) + gold["zpe"]
    opts = LobpcgOpts(n_iter=max_iter)
    if form == "mixed":
        model, tree, x0 = make_problem("c1", 10, 8)
        ms = MixedEigensolver(ctx, tree, model, D=8, k=10, low="fp32", hi="f64_f32")
        ms.load_block(x0)
        s = ms.lo
    else:
        s, model, tree = make_solver(api, ctx, "c1", form, 10, 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.lobpcg_start(opts)
    prev = None
    for it in range(max_iter):
        s.lobpcg_step()
        lam = np.sort(s.lam_d.cpu().numpy() + s.zpe)
        if np.max(np.abs(lam - ref)) <= tol and (form != "mixed" or s is ms.hi):
            return it + 1, time.perf_counter() - t0, float(np.max(np.abs(lam - ref)))
        if form == "mixed" and s is ms.lo and prev is not None and np.max(np.abs(lam - prev)) < switch_tol:
            ms.promote()
            s = ms.hi
        prev = lam
    return None


def time_to_solution_block(args, api):
    """Time-to-all-states entries of the bench line: the 6-mode workload
    against its exact levels, every form; and, unless --no-tts-c3, the
    12-mode fork-4 workload (k=84, D=40), plain FP64 against the mixed form,
    both against the plain FP64 run's own iterate --tts-c3-ref (the FP64 GPU
    path is pinned to the oracle on the small workloads)."""
    out = {"c1": {"workload": "6-mode coupled oscillators, MPS, D=8, k=10 (exact reference)", "tol_cm-1": 1e-3}}
    for form in ("fp64", "fp32", "f64_f32", "mixed"):
        c = api.Context(0, workspace_bytes=1 << 30)
        hit = time_to_all_states(api, c, form)
        out["c1"][form] = None if hit is None else {"iters": hit[0], "seconds": round(hit[1], 3),
                                                    "max_err_cm-1": hit[2]}
        c.close()
    if not args.no_tts_c3:
        a = argparse.Namespace(**vars(args))
        a.workload, a.k, a.bond, a.ref_iters, a.tts_forms = "c3", 84, 40, args.tts_c3_ref, args.tts_c3_forms
        a.precision = "fp32"
        out["c3"] = tts_run(a)
    return out


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
    print(json.dumps(tts_run(args)), flush=True)


def tts_run(args):
    """Time to all states at 1e-3 cm^-1 on a large workload: plain FP64 block
    LOBPCG for ref_iters iterations (its last iterate is the reference), then
    each form of --tts-forms from the same initial block, timed from solver
    start.  Forms with an FP32-storage phase run it until the largest change
    of a Rayleigh quotient between iterations drops below switch_tol, then
    promote the block to FP64 storage; only iterations after that count as
    hits."""
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
    log(f"time to all states: {wl_name}, D={D}, k={k}, reference = plain FP64 iterate {args.ref_iters}")
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
    # the other forms from the same initial block:
    #   f64_f32      FP64 storage, bulk H contractions on FP32 matrix cores, S~ / Rayleigh quotients / RR in FP64
    #   mixed        FP32-storage LOBPCG, then promotion and f64_f32 iterations
    #   mixed_fp64   FP32-storage LOBPCG, then promotion and all-FP64 iterations
    for form in args.tts_forms.split(","):
        if form == "f64_f32":
            lo, hi = None, TTNEigensolver(ctx, tree, model, D=D, k=k, precision="f64_f32", ttno=ttno)
            hi.load_block(x0)
        else:
            hi_kind = {"mixed": "f64_f32", "mixed_fp64": "fp64"}[form]
            ms = MixedEigensolver(ctx, tree, model, D=D, k=k, low=args.precision, ttno=ttno, hi=hi_kind)
            ms.load_block(x0)
            lo, hi = ms.lo, ms.hi
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cur = lo if lo is not None else hi
        cur.lobpcg_start(LobpcgOpts(n_iter=args.ref_iters))
        traj, prev, switched = [], None, None
        for it in range(args.ref_iters):
            cur.lobpcg_step()
            lam = np.sort(cur.lam_d.cpu().numpy() + cur.zpe)
            traj.append((time.perf_counter() - t0, lam, "lo" if cur is lo else "fp64"))
            log(f"  {form} iteration {it + 1} ({traj[-1][2]}): {traj[-1][0]:.1f} s, "
                f"max err {np.max(np.abs(lam - ref)):.5f}")
            if np.max(np.abs(lam - ref)) <= 1e-3 and cur is hi:
                break
            if cur is lo and prev is not None and np.max(np.abs(lam - prev)) < args.switch_tol:
                ms.promote()
                cur = hi
                switched = it + 1
            prev = lam
        del lo, hi
        if form != "f64_f32":
            del ms
        mi, mt = first_hit(traj)
        out[form] = {"switch_at_iter": switched, "iters": mi, "seconds": mt,
                     "s_per_iter": round(traj[-1][0] / len(traj), 3),
                     "max_err_per_iter": [round(float(np.max(np.abs(t[1] - ref))), 5) for t in traj]}
        if form != "f64_f32":
            out[form]["low"] = args.precision
        if pt and mt:
            out[form]["speedup_vs_plain"] = round(pt / mt, 3)
    ctx.close()
    return out


def e1_experiment(args):
    """The paper's 64-mode coupled-oscillator reproduction (Sec. III.A): the
    lowest 30 states at D=5 by 6 block-LOBPCG iterations on the MPS and on the
    T tree of Appendix B (8 harmonic-oscillator functions per mode), plain
    FP64; absolute errors against the normal-mode levels stored with the
    oracle runs (tests/golden/e1_oracle_runs.json)."""
    import torch
    import workloads as wl
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import LobpcgOpts, TTNEigensolver

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "e1_oracle_runs.json")))
    exact = np.array(gold["exact"][:args.e1_k]) + gold["zpe"]
    m = wl.paper_64d_model()
    out = {"experiment": "64-mode coupled oscillators (Sec. III.A)", "D": args.e1_bond, "k": args.e1_k,
           "iterations": args.e1_iters, "basis": "8 harmonic-oscillator functions per mode (FBR)", "runs": {}}
    out["ttno"] = args.ttno_method
    for name in ("mps", "ttree"):
        ctx = api.Context(0, workspace_bytes=2 << 30)
        tree = wl.paper_topology(name, m.dims)
        bonds = wl.bond_dims(tree, args.e1_bond)
        x0 = wl.initial_block(tree, bonds, m.omega, m.dims, args.e1_k, 117)
        gt = api.Tree(tree.parent, tree.phys)
        ttno = api.sop_build(gt, tree.mode, m.omega, m.dims, m.monomials, m.coefs, method=args.ttno_method)
        s = TTNEigensolver(ctx, tree, m, D=args.e1_bond, k=args.e1_k, precision="fp64", ttno=ttno)
        s.load_block(x0)
        lam0 = s.rayleigh_quotients(s.B, list(range(args.e1_k))).cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam = np.sort(s.lobpcg(LobpcgOpts(n_iter=args.e1_iters, shift=float(lam0.min()) - 1.0)))
        dt = time.perf_counter() - t0
        err = lam - exact
        hist = [float(np.max(np.abs(np.sort(h["lam"]) - exact))) for h in s.history]
        out["runs"][name] = {"seconds": round(dt, 2), "max_abs_err": float(np.max(np.abs(err))),
                             "mean_abs_err": float(np.mean(np.abs(err))), "min_err": float(err.min()),
                             "states_below_1e-2": int(np.sum(np.abs(err) < 1e-2)),
                             "abs_err_per_state": [round(float(e), 6) for e in err],
                             "max_err_per_iteration": [round(e, 5) for e in hist],
                             "ttno_max_bond": int(max(s.M))}
        print(f"  {name}: {dt:.1f} s, max err {np.max(np.abs(err)):.4g}, "
              f"{out['runs'][name]['states_below_1e-2']} of {args.e1_k} states below 1e-2", file=sys.stderr, flush=True)
        del s
        ctx.close()
    print(json.dumps(out), flush=True)


def topology_experiment(args):
    """The paper's topology comparison (Table tab:ch3cn_summary) on the
    12-mode synthetic force field (seed 3), 84 states: for every topology of
    Appendix B, block LOBPCG at D = --topo-bonds (5 iterations each, the
    paper's LOBPCG stage count) in the mixed form's f64_f32 arithmetic, timed;
    errors against a reference from the fork-4 comb at D=40 (mixed form, run
    to --topo-ref-iters iterations), all values variational upper bounds."""
    import torch
    import workloads as wl
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import LobpcgOpts, MixedEigensolver, TTNEigensolver

    m = wl.make_config_model("c3")
    k = 84
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    ctx = api.Context(0, workspace_bytes=8 << 30)
    tree = wl.fork_tree(m.dims, 4, 1)
    x0 = wl.initial_block(tree, wl.bond_dims(tree, 40), m.omega, m.dims, k, m.seed + 17)
    ms = MixedEigensolver(ctx, tree, m, D=40, k=k, low="fp32", hi="f64_f32")
    ms.load_block(x0)
    cur = ms.lo
    cur.lobpcg_start(LobpcgOpts(n_iter=args.topo_ref_iters))
    t0 = time.perf_counter()
    for it in range(args.topo_ref_iters):
        cur.lobpcg_step()
        if cur is ms.lo and it + 1 == 10:
            ms.promote()
            cur = ms.hi
    ref = np.sort(cur.lam_d.cpu().numpy() + cur.zpe)
    log(f"reference (fork-4, D=40, {args.topo_ref_iters} iterations): {time.perf_counter() - t0:.1f} s")
    del ms, cur
    ctx.close()
    out = {"experiment": "topology comparison (Table tab:ch3cn_summary shape)", "workload": "c3 seed 3, k=84",
           "reference": f"fork-4 comb, D=40, mixed form, {args.topo_ref_iters} LOBPCG iterations", "runs": {}}
    for D in [int(x) for x in args.topo_bonds.split(",")]:
        for name in ("mps", "ttree", "leafonly", "fork3", "fork4", "fork6", "t3ns"):
            ctx = api.Context(0, workspace_bytes=8 << 30)
            tree = wl.paper_topology(name, m.dims)
            x0 = wl.initial_block(tree, wl.bond_dims(tree, D), m.omega, m.dims, k, m.seed + 17)
            s = TTNEigensolver(ctx, tree, m, D=D, k=k, precision="f64_f32")
            s.load_block(x0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lam = np.sort(s.lobpcg(LobpcgOpts(n_iter=args.topo_iters)))
            dt = time.perf_counter() - t0
            err = lam - ref
            out["runs"][f"{name}_D{D}"] = {"topology": name, "D": D, "seconds": round(dt, 2),
                                           "mean_abs_err": round(float(np.mean(np.abs(err))), 4),
                                           "max_abs_err": round(float(np.max(np.abs(err))), 4),
                                           "min_signed_err": round(float(err.min()), 4),
                                           "ttno_max_bond": int(max(s.M))}
            log(f"  {name} D={D}: {dt:.1f} s, mean |err| {np.mean(np.abs(err)):.4f}, max {np.max(np.abs(err)):.4f}")
            del s
            ctx.close()
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


def grow_experiment(args):
    """The paper's two-stage schedule on the 12-mode force field (the
    acetonitrile stand-in, Sec. III.B): block LOBPCG at maximum bond D_lo
    (ALS preconditioner 2 sweeps, MINRES <= 10), then block inverse iteration
    (clusters below 5 cm^-1, 1 ALS sweep, MINRES <= maxiter) -- once with every
    bond grown to D_hi by the residual-driven expansion, once at D_lo from the
    same states.  Reports each stage's time and the Rayleigh quotients (all
    variational: lower is better)."""
    import torch
    from paper_2512_15875_amd import ttn as api
    from paper_2512_15875_amd.solver import IIOpts, LobpcgOpts, TTNEigensolver, build_ttno

    k = args.k or 84
    model, tree, x0 = make_problem("c3", k, args.grow_lo)
    ctx = api.Context(0, workspace_bytes=8 << 30)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    W = build_ttno(api.Tree(tree.parent, tree.phys), tree, model)
    s = TTNEigensolver(ctx, tree, model, D=args.grow_lo, k=k, precision="fp64", ttno=W)
    s.load_block(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.lobpcg(LobpcgOpts(n_iter=args.grow_lobpcg, shift=None),
             log=lambda r: log(f"  LOBPCG D={args.grow_lo} {r['iter'] + 1}: {time.perf_counter() - t0:.1f} s"))
    ctx.sync()
    t_lob = time.perf_counter() - t0
    lam_lob = np.sort(s.lam_d.cpu().numpy() + s.zpe)
    snap = [s.B.t[u][:k].clone() for u in range(s.gt.n)]
    lam_snap = s.lam_d.clone()
    opts = IIOpts(n_iter=args.grow_ii, minres_maxiter=args.grow_maxiter, minres_rtol=1e-10)
    out = {"experiment": "LOBPCG at D_lo, bond growth, inverse iteration at D_hi (Sec. III.B schedule)",
           "workload": f"c3 12-mode quartic force field, fork-4 comb, k={k}",
           "lobpcg": {"D": args.grow_lo, "iters": args.grow_lobpcg, "seconds": round(t_lob, 2)}}
    res = {}
    for name, D in (("ii_grown", args.grow_hi), ("ii_same_bond", args.grow_lo)):
        for u in range(s.gt.n):
            s.B.t[u][:k].copy_(snap[u])
        s.lam_d.copy_(lam_snap)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tgt = s
        t_grow = 0.0
        if D != args.grow_lo:
            tgt = s.grow(D, seed=77)
            ctx.sync()
            t_grow = time.perf_counter() - t1
            log(f"  grown to D={D}: {t_grow:.1f} s")
        theta = tgt.inverse_iteration(opts, log=lambda r: log(f"  {name} II {r['iter'] + 1}: "
                                                                f"{time.perf_counter() - t1:.1f} s"))
        ctx.sync()
        dt = time.perf_counter() - t1
        res[name] = np.sort(theta)
        out[name] = {"D": D, "seconds": round(dt, 2), "growth_seconds": round(t_grow, 2), "iters": args.grow_ii,
                     "minres_maxiter": args.grow_maxiter,
                     "mean_drop_from_lobpcg_cm-1": round(float(np.mean(lam_lob - res[name])), 5),
                     "max_drop_from_lobpcg_cm-1": round(float(np.max(lam_lob - res[name])), 5)}
        if tgt is not s:
            del tgt
    out["mean_lambda_grown_minus_same_bond_cm-1"] = round(float(np.mean(res["ii_grown"] - res["ii_same_bond"])), 5)
    out["states_lower_when_grown"] = int(np.sum(res["ii_grown"] < res["ii_same_bond"] - 1e-6))
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
    # per launch: the three products of the staged path, and the compulsory
    # bytes (bra and ket tensors, two environments in, one out, per pair)
    fl = 2.0 * Dn ** 4 * 3 * n
    by = 4.0 * n * (2 * Dn ** 3 + 3 * Dn ** 2)
    print(json.dumps({"ienv_probe": f"3-leg node, bonds {Dn}, {ks} states, {n} pairs, FP32",
                      "kernels": {"ienv3_kernel": {"algorithmic_flop_per_launch": fl,
                                                   "algorithmic_bytes_per_launch": by}}}), flush=True)


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
    # U2 compulsory bytes of the step: per environment update (u -> parent),
    # with and without the operator, the 3k node tensors once, every pair's
    # incoming and outgoing environments, the site operator once
    es = 8 if args.precision in ("fp64", "f64_f32") else 4
    n_pairs = len(ia)
    u2 = 0.0
    for (u, p) in s.up_edges:
        ch = [c for c in s.gt.nbrs(u) if c != p]
        a_u = float(np.prod(s.B.legdims(u)))
        for with_op in (True, False):
            m_of = (lambda c: max(1, s.M[c])) if with_op else (lambda c: 1)
            env_in = sum(s.bonds[c] * m_of(c) * s.bonds[c] for c in ch)
            env_out = s.bonds[u] * m_of(u) * s.bonds[u]
            u2 += es * (m * a_u + n_pairs * (env_in + env_out) + (s.Wd[u].numel() if with_op else 0))
    print(json.dumps({"gram_probe": f"c2, D={D}, k={k}, {len(ia)} pairs", "u2_alg_bytes_step": u2,
                      "kernels": out}), flush=True)


def heff_probe(args):
    """The headline U1 alone: heff_apply_block with the TTNO at the headline
    node for k states (random FP32 inputs at the node's exact shapes: the
    same plan, kernels and grids as the bench step's MINRES products there),
    repeated --probe-reps times between the markers.  Prints the per-kernel
    algorithmic flops and bytes per launch, for rocprofv3 counter passes,
    which take a short program."""
    import torch
    from paper_2512_15875_amd import ttn as api

    k = args.k or (50 if args.workload == "c2" else 84)
    D = args.bond or (24 if args.workload == "c2" else 40)
    ctx = api.Context(0, workspace_bytes=8 << 30)
    api.autotune(ctx, args.autotune)
    s, model, tree = make_solver(api, ctx, args.workload, args.precision, k, D)
    u = headline_nodes(s, args.workload)[0]
    nb = s.gt.nbrs(u)
    envs = api.Envs(ctx, s.gt, k, s.bonds, s.M, s.bonds, s.sdt, edges=[api.dslot(s.gt, c, u) for c in nb])
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    for c in nb:
        e = envs.get(c, u)
        e.copy_(torch.randn(e.shape, generator=g, device="cuda", dtype=e.dtype))
    n_loc = int(np.prod(s.B.legdims(u)))
    X = torch.randn(k, n_loc, generator=g, device="cuda", dtype=s.tdt)
    Y = torch.empty_like(X)
    shift = torch.full((k,), -837.0, dtype=torch.float64, device="cuda")
    call = lambda: api.heff_apply_block(ctx, s.gt, s.op, envs, u, k, X, Y, shift=shift, compute=s.compute)
    call()  # plan and tables (and, with --autotune, the measured tile choice)
    ctx.sync()
    if args.autotune:
        for line in api.autotune(ctx, None).splitlines():
            if line.startswith(f"heff:{u}:1"):
                print("  tuned " + line, file=sys.stderr)
    for _ in range(20):  # steady clocks before the measured calls
        call()
    ctx.sync()
    mark = torch.zeros(MARKER_N, dtype=torch.float64, device="cuda")
    api.vec_scale(ctx, mark, 1.0, mark)
    api.probe_heff(ctx, [u])
    api.profile(ctx, True)
    for _ in range(args.probe_reps):
        call()
    n_calls, fl, ms = api.probe_report(ctx)
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    api.vec_scale(ctx, mark, 1.0, mark)
    ctx.sync()
    roof, by_kernel = stage_roofline(rep, args.precision)
    kern = {kn: {"launches": d["launches"], "avg_ms": round(d["ms"] / d["launches"], 5),
                 "algorithmic_flop_per_launch": d["flops"] / d["launches"],
                 "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
                 "tflop_per_s": round(d["flops"] / (d["ms"] * 1e-3) / 1e12, 2),
                 "stage_shapes_MNK_items": sorted(d["shapes"])} for kn, d in by_kernel.items()}
    # U1 compulsory bytes per call: k (|X| + |Y|), every state's incoming
    # environments, the site operator
    es = X.element_size()
    u1_bytes = es * (2 * k * n_loc + sum(envs.get(c, u).numel() for c in nb) + s.Wd[u].numel())
    print(json.dumps({"heff_probe": f"{args.workload} node {u}, D={D}, k={k}, {args.precision}, {n_calls} calls",
                      "tflop_per_s": round(fl / (ms * 1e-3) / 1e12, 2), "ms_per_call": round(ms / n_calls, 4),
                      "gflop_per_call": round(fl / n_calls / 1e9, 3), "calls": n_calls,
                      "u1_alg_bytes_per_call": u1_bytes, "kernels": kern}), flush=True)


def trace_summary(path: str, kernel: str):
    """Summary of a rocprofv3 kernel-trace CSV (kernel_trace.csv of
    --kernel-trace) of a default bench run: the bench brackets its timed
    LOBPCG iterations and then its extra profiled iteration with vec_scale
    launches over MARKER_N doubles (a grid no other launch uses).  Prints the
    kernel mix of the profiled iteration (between the third and fourth
    markers), the mean duration of the kernels named by the prefix `kernel`
    over the timed iterations (between the first two), and the whole trace's
    top kernels."""
    import csv
    rows = list(csv.DictReader(open(path)))
    rec = []
    for r in rows:
        name = r.get("Kernel_Name", "")
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        gx = int(r.get("Grid_Size_X", r.get("Grid_Size", "0")) or 0)
        rec.append((t0, t1, name, gx))
    rec.sort()
    # the library names the unit-stride-k tiles by their FP32 instance without the storage type
    short = lambda k: k.replace("void ttn::", "").replace("ttn::", "").split("(")[0].replace(", float>", ">")
    marker_grid = -(-MARKER_N // 256) * 256
    marks = [i for i, (_, _, n, gx) in enumerate(rec) if "vscale_kernel" in n and gx == marker_grid]

    def table(sel, title):
        by = {}
        for t0, t1, n, _ in sel:
            a = by.setdefault(short(n), [0, 0.0])
            a[0] += 1
            a[1] += (t1 - t0) * 1e-6
        tot = sum(v[1] for v in by.values())
        print(f"{title}: {sum(v[0] for v in by.values())} dispatches, {tot:.1f} ms of kernel time.\n")
        print("| kernel | launches | total ms | avg us | share |")
        print("|---|---|---|---|---|")
        for n, (c, ms) in sorted(by.items(), key=lambda kv: -kv[1][1])[:20]:
            print(f"| {n} | {c} | {ms:.1f} | {1e3 * ms / c:.1f} | {ms / tot:.3f} |")
        print()

    if len(marks) >= 4:
        table(rec[marks[2] + 1:marks[3]], "Kernels in the profiled iteration")
        timed = [x for x in rec[marks[0] + 1:marks[1]] if short(x[2]).startswith(kernel)]
        by = {}
        for t0, t1, n, gx in timed:
            by.setdefault((short(n), gx), []).append((t1 - t0) * 1e-3)
        print(f"Kernels named {kernel}* over the timed iterations (between the first two markers), by grid "
              f"(the launches of one contraction stage share a grid):\n")
        print("| kernel | grid (threads) | launches | avg us |")
        print("|---|---|---|---|")
        for (n, gx), d in sorted(by.items(), key=lambda kv: -sum(kv[1])):
            print(f"| {n} | {gx} | {len(d)} | {np.mean(d):.1f} |")
        print()
    else:
        print(f"({len(marks)} marker launches found; the region tables need four)\n")
    table(rec, "Whole trace (setup and warm-up included)")


def pmc_summary(out: str, probe: str = "heff"):
    """Markdown summary of rocprofv3 counter passes over `bench.py
    --<probe>-probe` (directories out/<probe>_p*/ with
    <probe>_counter_collection.csv, the probe's JSON line in out/<probe>_p1.log)
    and of the copy calibration (out/copy_FETCH_SIZE/, out/copy_WRITE_SIZE/):
    per kernel, the mean per dispatch of every counter, HBM bytes from
    FETCH_SIZE / WRITE_SIZE scaled by the copy, MFMA utilisation and executed
    MFMA flops; the whole probe's measured bytes against its compulsory
    bytes; then one traffic|kernel|gemm hash|measured bytes|algorithmic bytes
    line per GEMM kernel."""
    import csv
    import glob
    per = {}
    region = {}  # counter -> sum over the dispatches between the probe's two markers
    marker_grid = -(-MARKER_N // 256) * 256
    for f in sorted(glob.glob(os.path.join(out, f"{probe}_p*", f"{probe}_counter_collection.csv"))):
        rows = list(csv.DictReader(open(f)))
        for r in rows:
            per.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        marks = sorted(int(r["Start_Timestamp"]) for r in rows
                       if "vscale_kernel" in r["Kernel_Name"] and int(r["Grid_Size"]) == marker_grid)
        if len(marks) >= 2:
            for r in rows:
                if marks[0] < int(r["Start_Timestamp"]) < marks[1]:
                    region[r["Counter_Name"]] = region.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    cal = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        f = os.path.join(out, f"copy_{c}", "copy_counter_collection.csv")
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(f)) if "copyBuffer" in r["Kernel_Name"]]
        cal[c] = (256 << 20) / (float(np.median(vals)) * 1024)  # bytes per KiB reported, for a 256 MiB copy
    info = None
    for line in open(os.path.join(out, f"{probe}_p1.log")):
        if line.startswith('{"' + probe + '_probe"'):
            info = json.loads(line)
    kinfo = (info or {}).get("kernels", {})
    # the library names the unit-stride-k tiles by their FP32 instance without the storage type
    short = lambda k: k.replace("void ttn::", "").split("(")[0].replace(", float>", ">")

    def lookup(kn):  # the probe names fused kernels without their template arguments
        return kinfo.get(kn) or kinfo.get(kn.split("<")[0])

    print(f"Copy calibration (256 MiB device copy): FETCH_SIZE x {cal['FETCH_SIZE']:.3f} KiB, "
          f"WRITE_SIZE x {cal['WRITE_SIZE']:.3f} KiB = bytes\n")
    print("| kernel | dispatches | HBM read MB | HBM write MB | algorithmic MB | traffic / algorithmic | MFMA busy "
          "(of GRBM_GUI_ACTIVE x 1024 SIMDs) | MFMA flops executed / algorithmic |")
    print("|---|---|---|---|---|---|---|---|")
    lines = []
    h = gemm_source_hash()
    tot_bytes = (region.get("FETCH_SIZE", 0.0) * cal["FETCH_SIZE"] +
                 region.get("WRITE_SIZE", 0.0) * cal["WRITE_SIZE"]) * 1024
    for name, cs in per.items():
        kn = short(name)
        m = {c: float(np.mean(v)) for c, v in cs.items()}
        nd = len(next(iter(cs.values())))
        rd = m.get("FETCH_SIZE", 0.0) * 1024 * cal["FETCH_SIZE"]
        wr = m.get("WRITE_SIZE", 0.0) * 1024 * cal["WRITE_SIZE"]
        pk = lookup(kn)
        if pk is None:
            continue
        alg = pk["algorithmic_bytes_per_launch"]
        alg_fl = pk["algorithmic_flop_per_launch"]
        util = (m["SQ_VALU_MFMA_BUSY_CYCLES"] / (m["GRBM_GUI_ACTIVE"] / 8 * 1024)
                if m.get("GRBM_GUI_ACTIVE") else float("nan"))
        exe = m.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) * 512
        print(f"| {kn} | {nd} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {alg / 1e6:.1f} | "
              f"{(rd + wr) / alg if rd + wr else float('nan'):.3f} | {util:.3f} | "
              f"{exe / alg_fl if alg_fl else float('nan'):.3f} |")
        if rd + wr and (kn.startswith("ogemm") or kn.startswith("relayout")):
            lines.append(f"traffic|{kn}|{h}|{rd + wr:.6e}|{alg:.6e}")
    # the measured region (between the probe's markers) of the FETCH_SIZE and
    # WRITE_SIZE passes: the probe's calls, nothing of its set-up or warm-up
    if info and tot_bytes:
        if "u1_alg_bytes_per_call" in info:
            per_call = tot_bytes / info["calls"]
            print(f"\nWhole U1 call: measured {per_call / 1e6:.1f} MB per call against the compulsory "
                  f"{info['u1_alg_bytes_per_call'] / 1e6:.1f} MB (k (|X| + |Y|) + the k states' environments + W): "
                  f"{per_call / info['u1_alg_bytes_per_call']:.2f}x")
            lines.append(f"u1call|{h}|{per_call:.6e}|{info['u1_alg_bytes_per_call']:.6e}")
        if "u2_alg_bytes_step" in info:
            print(f"\nWhole Gram step: measured {tot_bytes / 1e9:.2f} GB against the compulsory U2 bytes "
                  f"{info['u2_alg_bytes_step'] / 1e9:.2f} GB (node tensors once, every pair's environments in and "
                  f"out, W once, per update with and without the operator): {tot_bytes / info['u2_alg_bytes_step']:.2f}x")
    print("\nOther counters, mean per dispatch:\n")
    for name, cs in per.items():
        kn = short(name)
        if lookup(kn) is None:
            continue
        print(f"* {kn}: " + ", ".join(f"{c} {np.mean(v):.4g}" for c, v in sorted(cs.items())))
    print("\nGEMM source hash (sha256[:16] of csrc/gemm.hip): " + h + "\n")
    print("```")
    for l in lines:
        print(l)
    print("```")


def cpu_baseline(api, ctx, s, u: int, k: int, reps: int = 5):
    """The FP64 oracle timed on the host at the headline node u: U1 = K2
    (one state's H_eff apply) and U2 = K1 (one pair's environment update
    u -> parent(u)), each on all the BLAS threads the process has and on one
    thread, median of `reps` samples.  Inputs are random at the node's exact
    shapes (bonds, operator bonds); flops are the library's algorithmic counts
    of the same operations, so the rates compare with the GPU's."""
    from threadpoolctl import threadpool_limits

    from oracle import ttn as ottn

    tree = s.wtree
    nb = tree.neighbours(u)
    v = tree.parent[u]
    rng = np.random.default_rng(7)
    edge = lambda c: u if c == tree.parent[u] else c
    Db = [s.bonds[edge(c)] for c in nb]
    W = rng.normal(size=tuple(s.M[edge(c)] for c in nb) + (1, 1))
    X = rng.normal(size=tuple(Db) + (1,))
    A2 = rng.normal(size=tuple(Db) + (1,))
    E = {c: rng.normal(size=(Db[i], s.M[edge(c)], Db[i])) for i, c in enumerate(nb)}
    envs = api.Envs(ctx, s.gt, 1, s.bonds, s.M, s.bonds, s.sdt, edges=[api.dslot(s.gt, c, u) for c in s.gt.nbrs(u)])
    f_u1 = api.flops_heff(s.gt, s.op, envs, u, 1)
    f_u2 = api.flops_env(s.gt, s.op, s.B, s.B, u, v)
    ein2 = {c: E[c] for c in nb if c != v}
    units = {"U1": (lambda: ottn.heff_apply(tree, u, W, X, E), f_u1),
             "U2": (lambda: ottn.env_update(tree, u, v, X, W, A2, ein2), f_u2)}
    all_threads = blas_threads()
    out = {}
    for name, (fn, fl) in units.items():
        for label, nt in (("all", all_threads), ("one", 1)):
            with threadpool_limits(limits=nt, user_api="blas"):
                fn()  # warm
                ts = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    fn()
                    ts.append(time.perf_counter() - t0)
            med = float(np.median(ts))
            out[f"{name}_{label}"] = {"gflop_per_s": round(fl / med / 1e9, 3), "median_s": round(med, 4),
                                      "threads": nt, "gflop": round(fl / 1e9, 3)}
    u1 = out["U1_all"]
    return {"value": u1["gflop_per_s"], "unit": "GFLOP/s", "cores": all_threads, "kind": "oracle",
            "sample": f"FP64 NumPy oracle at the headline node {u} (n_loc={int(np.prod(Db))}): U1 = one state's "
                      f"H_eff apply, U2 = one pair's environment update {u}->{v}; median of {reps} samples each on "
                      f"{all_threads} BLAS threads and on 1; value = U1 on {all_threads} threads",
            "affinity_cores": len(os.sched_getaffinity(0)), "blas": blas_vendor(), **out}


def blas_vendor():
    try:
        from threadpoolctl import threadpool_info
        return ",".join(sorted({f"{i.get('internal_api')}" for i in threadpool_info() if i.get("user_api") == "blas"}))
    except Exception:
        return "unknown"


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
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64", "bf16", "f64_f32"])
    ap.add_argument("--workload", default="c2", choices=["c2", "c3"])
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--bond", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tts", action="store_true")
    ap.add_argument("--no-tts-c3", action="store_true", help="skip the 12-mode time-to-all-states comparison")
    ap.add_argument("--tts-c3-ref", type=int, default=34)
    ap.add_argument("--tts-c3-forms", default="mixed")
    ap.add_argument("--calibrate-copy", action="store_true", help="only run the copy kernel used to scale counters")
    ap.add_argument("--workspace-gb", type=float, default=8.0,
                    help="library workspace of the bench step (stage intermediates; bounds the items per launch)")
    ap.add_argument("--gram-probe", action="store_true", help="only the Gram step, for counter passes")
    ap.add_argument("--ienv-probe", action="store_true",
                    help="only the fused identity overlap environment at a 24x24x24 node, for counter passes")
    ap.add_argument("--probe-pairs", type=int, default=20000)
    ap.add_argument("--probe-reps", type=int, default=5)
    ap.add_argument("--ii", action="store_true", help="run the inverse-iteration experiment instead")
    ap.add_argument("--e1", action="store_true", help="the paper's 64-mode coupled-oscillator reproduction")
    ap.add_argument("--e1-k", type=int, default=30)
    ap.add_argument("--ttno-method", default="svd", choices=["svd", "state_diagram"],
                    help="operator compiler of the --e1 runs")
    ap.add_argument("--e1-bond", type=int, default=5)
    ap.add_argument("--e1-iters", type=int, default=6)
    ap.add_argument("--topologies", action="store_true", help="the 12-mode topology comparison")
    ap.add_argument("--topo-bonds", default="12,20")
    ap.add_argument("--topo-iters", type=int, default=5)
    ap.add_argument("--topo-ref-iters", type=int, default=30)
    ap.add_argument("--grow", action="store_true",
                    help="LOBPCG at --grow-lo, bond growth, inverse iteration at --grow-hi (c3)")
    ap.add_argument("--grow-lo", type=int, default=12)
    ap.add_argument("--grow-hi", type=int, default=20)
    ap.add_argument("--grow-lobpcg", type=int, default=5)
    ap.add_argument("--grow-ii", type=int, default=5)
    ap.add_argument("--grow-maxiter", type=int, default=10000)
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
    ap.add_argument("--tts-forms", default="f64_f32,mixed,mixed_fp64",
                    help="forms compared with plain FP64 in --tts: f64_f32, mixed (FP32 storage, then f64_f32), "
                         "mixed_fp64 (FP32 storage, then all-FP64)")
    ap.add_argument("--gemm-hash", action="store_true", help="print the GEMM source hash and exit")
    ap.add_argument("--heff-probe", action="store_true", help="run only the headline heff_apply_block calls")
    ap.add_argument("--trace-summary", default=None, help="summarise a rocprofv3 kernel_trace.csv and exit")
    ap.add_argument("--trace-kernel", default="ogemm_tn_kernel", help="kernel-name prefix timed over the timed iterations")
    ap.add_argument("--pmc-summary", default=None,
                    help="summarise rocprofv3 counter passes over a probe (directory of the passes) and exit")
    ap.add_argument("--pmc-probe", default="heff", choices=["heff", "gram", "ienv"],
                    help="which probe the counter passes ran (--heff-probe, --gram-probe, --ienv-probe)")
    args = ap.parse_args()
    if args.graphs and args.warmup < 2:
        args.warmup = 2  # first step runs eagerly, the second captures: keep both untimed
    if args.gemm_hash:
        print(gemm_source_hash())
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.trace_kernel)
        return
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.pmc_probe)
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
    if args.heff_probe:
        heff_probe(args)
        return
    if args.ienv_probe:
        ienv_probe(args)
        return
    if args.ii:
        ii_experiment(args)
        return
    if args.grow:
        grow_experiment(args)
        return
    if args.e1:
        e1_experiment(args)
        return
    if args.topologies:
        topology_experiment(args)
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


def headline_nodes(s, workload: str):
    """The node class the metric is quoted on: the level-1 nodes of the binary
    tree (children of the root), or backbone node b2 (the root) of the fork-4
    comb."""
    return list(s.gt.children[s.root]) if workload == "c2" else [s.root]


def stage_roofline(rep, precision):
    """Roofline object of the kernel with the largest time among stage
    records `rep` (algorithmic flops and bytes per launch over its average
    launch duration, both from HIP events on the library stream)."""
    by_kernel = {}
    for key, st, kern, cnt, tms, fl, Mm, Nn, Kk, nz, by in rep:
        a = by_kernel.setdefault(kern, {"launches": 0, "ms": 0.0, "flops": 0.0, "bytes": 0.0, "shapes": set()})
        a["launches"] += cnt
        a["ms"] += tms
        a["flops"] += fl
        a["bytes"] += by
        a["shapes"].add((Mm, Nn, Kk, nz // max(cnt, 1)))
    kern, d = max(by_kernel.items(), key=lambda kv: kv[1]["ms"])
    tot = sum(v["ms"] for v in by_kernel.values())
    peak_tf = PEAK[precision]
    ridge = peak_tf * 1e12 / (HBM_TBS * 1e12)
    if d["flops"] / max(d["bytes"], 1.0) >= ridge:
        roof = {"bound": "mfma", "achieved": round(d["flops"] / (d["ms"] * 1e-3) / 1e12, 3), "peak": peak_tf,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(d["bytes"] / (d["ms"] * 1e-3) / 1e9, 1), "peak": HBM_TBS * 1e3,
                "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof.update({"kernel": kern, "launches": d["launches"], "avg_ms": round(d["ms"] / d["launches"], 5),
                 "algorithmic_flop_per_launch": d["flops"] / d["launches"],
                 "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
                 "stage_shapes_MNK_items": sorted(d["shapes"]),
                 "share_of_time": round(d["ms"] / tot, 3)})
    return roof, by_kernel


def run_bench(args, api, k, D, stream):
    import torch
    from paper_2512_15875_amd.solver import LobpcgOpts

    ctx = api.Context(0, workspace_bytes=int(args.workspace_gb * (1 << 30)), stream=stream)
    api.autotune(ctx, args.autotune)
    s, model, tree = make_solver(api, ctx, args.workload, args.precision, k, D)
    s.graphs = args.graphs
    s.lobpcg_start(LobpcgOpts(n_iter=args.warmup + args.steps + 2))
    hn = headline_nodes(s, args.workload)
    print(f"setup done: {tree.n} nodes, k={k}, D={D}, precision={args.precision}, headline nodes {hn}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        s.lobpcg_step()
        print(f"warmup step {i} done", file=sys.stderr, flush=True)
    ctx.sync()
    torch.cuda.synchronize()
    # Timed region: K whole LOBPCG iterations.  Every heff_apply_block call with
    # the operator at the headline nodes is bracketed by HIP events (the whole
    # call), and the stages of those calls by per-launch events; nothing else
    # is profiled.  Marker launches (vec_scale on MARKER_N doubles) bracket the
    # region for trace summaries.
    mark = torch.zeros(MARKER_N, dtype=torch.float64, device="cuda")
    api.vec_scale(ctx, mark, 1.0, mark)
    api.probe_heff(ctx, hn)
    api.profile_filter(ctx, [f"heff:{u}:1" for u in hn])
    api.profile(ctx, True)
    api.ctx_flops(ctx, reset=True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        s.lobpcg_step()
        print(f"step {i} done: lam0={s.history[-1]['lam'].min():.4f} max|r|={s.history[-1]['resid'].max():.3e}",
              file=sys.stderr, flush=True)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.vec_scale(ctx, mark, 1.0, mark)
    flops = api.ctx_flops(ctx)
    n_calls, call_fl, call_ms = api.probe_report(ctx)
    rep_u1 = api.profile_report(ctx)
    api.profile(ctx, False)
    api.profile_filter(ctx, [])
    api.probe_heff(ctx, [])
    ms = (t1 - t0) * 1e3 / args.steps
    value = call_fl / (call_ms * 1e-3) / 1e9
    roof, u1_kernels = stage_roofline(rep_u1, args.precision)
    stage_ms = sum(v["ms"] for v in u1_kernels.values())
    tr = measured_traffic(roof["kernel"])
    roof["traffic"] = None if tr is None else round(tr[0], 0)
    if tr is not None:
        roof["traffic_unit"] = "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
        roof["traffic_over_algorithmic_bytes"] = round(tr[0] / tr[1], 3)
    tc = measured_u1_call_traffic()
    if tc is not None:
        roof["u1_call_traffic_bytes"] = round(tc[0], 0)
        roof["u1_call_traffic_over_compulsory"] = round(tc[0] / tc[1], 2)
    for kern, d in sorted(u1_kernels.items(), key=lambda kv: -kv[1]["ms"]):
        print(f"  U1 kernel {kern}: {d['launches']} launches {d['ms']:.1f} ms "
              f"{d['flops'] / (d['ms'] * 1e-3) / 1e12:.1f} TFLOP/s shapes {sorted(d['shapes'])}", file=sys.stderr)
    print(f"headline H_eff applies: {n_calls} calls, {call_ms:.1f} ms ({stage_ms:.1f} ms in stages), "
          f"{value / 1e3:.1f} TFLOP/s", file=sys.stderr, flush=True)

    # one more step with every stage profiled (outside the timed region): the
    # step's kernel mix, its dominant kernel and all H_eff applies
    api.vec_scale(ctx, mark, 1.0, mark)
    api.profile(ctx, True)
    s.lobpcg_step()
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    api.vec_scale(ctx, mark, 1.0, mark)
    ctx.sync()
    step_roof, by_kernel = stage_roofline(rep, args.precision)
    tot_ms = sum(v["ms"] for v in by_kernel.values())
    for kern, d in sorted(by_kernel.items(), key=lambda kv: -kv[1]["ms"])[:8]:
        print(f"  step kernel {kern}: {d['launches']} launches {d['ms']:.1f} ms "
              f"{d['flops'] / (d['ms'] * 1e-3) / 1e12:.1f} TFLOP/s {d['bytes'] / (d['ms'] * 1e-3) / 1e9:.0f} GB/s",
              file=sys.stderr)
    qr_shapes = {}  # QR gauge moves by node matrix shape: launches, ms
    for key, st, kern, cnt, tms, *_r in rep:
        if key.startswith("qr:"):
            a = qr_shapes.setdefault(key[3:], [0, 0.0])
            a[0] += cnt
            a[1] += tms
    if qr_shapes:
        print("  QR moves by shape: " + ", ".join(f"{k} {v[0]} x {v[1] / v[0] * 1e3:.1f} us"
                                                  for k, v in sorted(qr_shapes.items(), key=lambda kv: -kv[1][1])),
              file=sys.stderr)
    heff_fl = heff_ms = 0.0
    by_depth = {}  # H_eff applies with the TTNO, by the node's distance from the root
    deep = {}  # their stage kernels at depth >= 3: (depth, kernel, (M, N, K, items)) -> ms, launches
    depth = {}
    for u in range(tree.n):
        d, v = 0, u
        while tree.parent[v] >= 0:
            v, d = tree.parent[v], d + 1
        depth[u] = d
    for key, st, kern, cnt, tms, fl, *_r in rep:
        parts = key.split(":")
        if parts[0] == "heff" and parts[2] == "1":
            heff_fl += fl
            heff_ms += tms
            a = by_depth.setdefault(depth[int(parts[1])], [0.0, 0.0, 0])
            a[0] += fl
            a[1] += tms
            a[2] += cnt
            if depth[int(parts[1])] >= 3:
                b = deep.setdefault((depth[int(parts[1])], kern, tuple(_r[:4])), [0.0, 0])
                b[0] += tms
                b[1] += cnt
    heff_levels = {str(d): {"ms": round(v[1], 2), "tflop_per_s": round(v[0] / (v[1] * 1e-3) / 1e12, 2) if v[1] else None,
                            "launches": v[2]} for d, v in sorted(by_depth.items())}
    print(f"  H_eff applies by depth: {heff_levels}", file=sys.stderr)
    for (dp, kn, shp), (tms, cnt) in sorted(deep.items(), key=lambda kv: -kv[1][0])[:16]:
        print(f"    depth {dp} {kn} MNK/items {shp}: {cnt} launches {tms:.2f} ms ({1e3 * tms / cnt:.1f} us each)",
              file=sys.stderr)
    peak_tf = PEAK[args.precision]

    workload_name = ("64-mode coupled oscillators + 200 cubic terms, binary leaf-only tree (127 nodes)"
                     if args.workload == "c2" else
                     "12-mode synthetic quartic force field (108 cubic + 191 quartic), fork-4 comb (16 nodes)")
    node_name = "level-1 nodes (24^3, operator bonds 63/42/36)" if args.workload == "c2" else "backbone node b2"
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
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16", "f64_f32": "f64/f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{workload_name}, D={D}, k={k}: heff_apply_block with the TTNO at the {node_name}, "
                               f"k={k} states per call, as issued inside K timed block-LOBPCG iterations (residual "
                               f"fit, ALS preconditioner 2 sweeps x MINRES<=10, 3k-subspace Gram + Rayleigh-Ritz, "
                               f"fitted recombination)",
                   "precision": args.precision, "autotune": bool(args.autotune), "graphs": bool(args.graphs)},
        "frac_of_peak": round(value / 1e3 / peak_tf, 4),
        "heff_headline": {"calls": n_calls, "call_ms": round(call_ms, 2), "stage_ms": round(stage_ms, 2),
                          "algorithmic_gflop": round(call_fl / 1e9, 2), "nodes": hn,
                          "gflop_per_call": round(call_fl / max(n_calls, 1) / 1e9, 3)},
        "step_rate": {"gflop_per_s": round(flops / (t1 - t0) / 1e9, 2),
                      "gflop_per_step": round(flops / args.steps / 1e9, 2)},
        "roofline": roof,
        "step_profile": {"note": "one extra profiled step after the timed region",
                         "dominant_kernel": step_roof,
                         "heff_all_nodes_tflop_per_s": round(heff_fl / (heff_ms * 1e-3) / 1e12, 2) if heff_ms else None,
                         "heff_all_nodes_frac_of_peak": round(heff_fl / (heff_ms * 1e-3) / 1e12 / peak_tf, 4)
                         if heff_ms else None,
                         "heff_by_depth": heff_levels,
                         "dispatches": int(sum(v["launches"] for v in by_kernel.values())),
                         "qr_ms": round(sum(v[1] for v in qr_shapes.values()), 2),
                         "contraction_ms": round(tot_ms, 1)},
    }
    if not args.no_tts:
        out["time_to_all_states"] = time_to_solution_block(args, api)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(api, ctx, s, hn[0], k)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
