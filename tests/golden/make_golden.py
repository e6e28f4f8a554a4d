"""Writes the stored oracle results used by the GPU solver tests.

Calls only the oracle and the seeded workload generators:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import exact, solvers, ttno  # noqa: E402


def c1_runs():
    m = wl.make_config_model("c1")
    tree = wl.mps_tree(m.dims, 2)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 8)
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, 10, m.seed + 17)
    lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
    shift = float(np.min(lam0)) - 837.0
    hist = []
    xs, lam = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=7, shift=shift), hist)
    out = {
        "cite": "oracle block LOBPCG (Alg. lobpcg_block) on the 6-mode coupled-oscillator workload, MPS rooted at "
                "site 3, D=8, k=10, 7 iterations, ALS preconditioner 2 sweeps / MINRES<=10 / rtol 1e-6, "
                "shift = min Rayleigh quotient - 837 cm^-1 (shifted frame: harmonic ZPE removed)",
        "zpe": m.zpe_harmonic,
        "shift": shift,
        "lam_history": [list(map(float, h["lam"])) for h in hist],
        "resid_history": [list(map(float, h["resid"])) for h in hist],
        "lam_final": list(map(float, lam)),
        "exact": list(map(float, exact.normal_mode_levels(m, 10))),
    }
    # LOBPCG (3 iterations) followed by inverse iteration (2 iterations)
    xs3, lam3 = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=3, shift=shift))
    iih = []
    # Alg. block_inverse_iteration as printed: the optional safeguard stays off
    xs_ii, theta = solvers.inverse_iteration(tree, W, xs3, lam3, solvers.IIOptions(n_iter=2, monotone=False), iih)
    out["lobpcg3_lam"] = list(map(float, lam3))
    out["ii2_lam_history"] = [list(map(float, h["lam"])) for h in iih]
    out["ii2_final_rr"] = list(map(float, theta))
    return out


def c1_grow_runs(D_lo=4, D_hi=8, n_sketch=6, sketch_seed=31):
    """c1: LOBPCG (3 iterations) at D_lo, every bond grown to D_hi by the
    residual-driven expansion (Sec. II.C.2; the D 12 -> 20 step of Sec. III.B),
    inverse iteration (2 iterations) at D_hi; and the same inverse iteration
    at D_lo for comparison.  Sketch matrices: workloads.sketch_matrices."""
    from oracle import expand
    m = wl.make_config_model("c1")
    tree = wl.mps_tree(m.dims, 2)
    W = ttno.build_ttno(tree, m)
    lo = wl.bond_dims(tree, D_lo)
    hi = [max(1, b) for b in wl.bond_dims(tree, D_hi)]
    x0 = wl.initial_block(tree, lo, m.omega, m.dims, 10, m.seed + 17)
    lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
    shift = float(np.min(lam0)) - 837.0
    xs, lam = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=3, shift=shift))
    om = wl.sketch_matrices(tree, n_sketch, sketch_seed)
    ys = [expand.expand_bonds(tree, W, solvers.normalized(tree, x), hi, om, n_sketch) for x in xs]
    iih = []
    _, theta = solvers.inverse_iteration(tree, W, ys, lam, solvers.IIOptions(n_iter=2, monotone=False), iih)
    _, theta_lo = solvers.inverse_iteration(tree, W, xs, lam, solvers.IIOptions(n_iter=2, monotone=False))
    return {"cite": f"c1 oracle: block LOBPCG 3 iterations at D={D_lo}, bonds grown to D={D_hi} by the residual-"
                    f"driven expansion (sketch {n_sketch} columns, workloads.sketch_matrices seed {sketch_seed}), "
                    f"block inverse iteration 2 iterations at D={D_hi} (and at D={D_lo} for comparison)",
            "zpe": m.zpe_harmonic, "shift": shift, "D_lo": D_lo, "D_hi": D_hi, "n_sketch": n_sketch,
            "sketch_seed": sketch_seed, "lobpcg3_lam": list(map(float, lam)),
            "grown_lam": list(map(float, solvers.rayleigh_quotients(tree, W, ys))),
            "ii_lam_history": [list(map(float, h["lam"])) for h in iih],
            "ii_final_rr": list(map(float, theta)), "ii_lo_final_rr": list(map(float, theta_lo)),
            "exact": list(map(float, exact.normal_mode_levels(m, 10)))}


def c3_cluster_runs(seed=7, D=8, k=12):
    """Fork-4 comb from the quartic-force-field generator at a small bond
    dimension, with a seed whose Rayleigh quotients after LOBPCG hold two
    clusters of two states (gaps below 5 cm^-1), so the in-cluster
    Rayleigh-Ritz step of Alg. block_inverse_iteration runs."""
    m = wl.make_config_model("c3", seed=seed)
    tree = wl.fork_tree(m.dims, 4, 1)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, D)
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, k, m.seed + 17)
    lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
    shift = float(np.min(lam0)) - 837.0
    hist = []
    xs, lam = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=3, shift=shift), hist)
    clusters = solvers.clusters_of(lam, 5.0)
    iih = []
    xs_ii, theta = solvers.inverse_iteration(tree, W, xs, lam, solvers.IIOptions(n_iter=2, monotone=False), iih)
    return {
        "cite": f"oracle block LOBPCG (Alg. lobpcg_block, 3 iterations) then block inverse iteration "
                f"(Alg. block_inverse_iteration, 2 iterations, clusters below 5 cm^-1, 1 ALS sweep, MINRES<=10000, "
                f"rtol 1e-10, safeguard off) and one global Rayleigh-Ritz, on the quartic force field of seed {seed} "
                f"(fork-4 comb rooted at backbone b2), D={D}, k={k}; shifted frame (harmonic ZPE removed)",
        "seed": seed, "D": D, "k": k,
        "zpe": m.zpe_harmonic,
        "shift": shift,
        "lam_history": [list(map(float, h["lam"])) for h in hist],
        "resid_history": [list(map(float, h["resid"])) for h in hist],
        "lobpcg3_lam": list(map(float, lam)),
        "clusters": [[int(j) for j in c] for c in clusters],
        "ii2_lam_history": [list(map(float, h["lam"])) for h in iih],
        "ii2_final_rr": list(map(float, theta)),
    }


def topology_runs(D=4, k=4, n_iter=2):
    """The 12-mode quartic force field (seed 3) on every topology of the
    paper's comparison (Appendix B), two oracle LOBPCG iterations at a small
    bond dimension: Rayleigh quotients and residual norms per iteration."""
    m = wl.make_config_model("c3")
    out = {"cite": f"oracle block LOBPCG (Alg. lobpcg_block), {n_iter} iterations, quartic force field seed 3 on "
                   f"the topologies of Appendix B, D={D}, k={k}; shifted frame",
           "D": D, "k": k, "zpe": m.zpe_harmonic, "runs": {}}
    for name in ("mps", "ttree", "leafonly", "fork3", "fork4", "fork6", "t3ns"):
        tree = wl.paper_topology(name, m.dims)
        W = ttno.build_ttno(tree, m)
        bonds = wl.bond_dims(tree, D)
        x0 = wl.initial_block(tree, bonds, m.omega, m.dims, k, m.seed + 17)
        lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
        shift = float(np.min(lam0)) - 837.0
        hist = []
        xs, lam = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=n_iter, shift=shift), hist)
        out["runs"][name] = {"shift": shift, "lam_history": [list(map(float, h["lam"])) for h in hist],
                             "resid_history": [list(map(float, h["resid"])) for h in hist],
                             "lam_final": list(map(float, lam))}
        print(name, "done", flush=True)
    return out


def e1_runs(D=5, k=8, n_iter=2, n_exact=30):
    """The paper's 64-mode bilinearly coupled oscillators (Sec. III.A,
    Eq. coupled_harmonic_oscillator: omega_j = sqrt(j/2), alpha = 0.1 for every
    pair), 8 harmonic-oscillator functions per mode, on the MPS and the T
    tree of Appendix B (arms of 22, 22 and 20 modes): two oracle LOBPCG
    iterations at D=5 for k=8 states, and the 30 lowest levels of the normal-mode
    closed form.  Preconditioner shift: lowest initial Rayleigh quotient - 1
    (the model's frequencies are of order 1)."""
    m = wl.paper_64d_model()
    out = {"cite": f"paper's 64-mode model (Sec. III.A), FBR d=8, oracle block LOBPCG {n_iter} iterations, D={D}, "
                   f"k={k}, MPS and T tree; normal-mode levels (shifted frame)",
           "D": D, "k": k, "zpe": m.zpe_harmonic, "exact": list(map(float, exact.normal_mode_levels(m, n_exact))),
           "runs": {}}
    for name in ("mps", "ttree"):
        tree = wl.paper_topology(name, m.dims)
        W = ttno.build_ttno(tree, m)
        bonds = wl.bond_dims(tree, D)
        x0 = wl.initial_block(tree, bonds, m.omega, m.dims, k, 117)
        lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
        shift = float(np.min(lam0)) - 1.0
        hist = []
        xs, lam = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=n_iter, shift=shift), hist)
        out["runs"][name] = {"shift": shift, "lam_history": [list(map(float, h["lam"])) for h in hist],
                             "resid_history": [list(map(float, h["resid"])) for h in hist],
                             "lam_final": list(map(float, lam)), "ttno_max_bond": int(max(ttno.ttno_bonds(tree, W)))}
        print(name, "done", flush=True)
    return out


def c4_member_runs(n_iter=2):
    """Two small members of the ensemble generator (seeds 4000 and 4001: the
    coupled-oscillator generator on a balanced binary tree and the quartic
    force field on a fork-4 comb; L, D, k drawn from the member's seed in
    reduced ranges): oracle block LOBPCG for n_iter iterations, then a
    restarted run of n_iter more from its states (a new shift from their
    Rayleigh quotients, no search directions carried over), as the ensemble
    driver runs a member twice."""
    members = wl.ensemble_members(2, seed0=4000, D_range=(4, 6), k_range=(3, 5), L_range=(8, 10))
    out = {"cite": f"oracle block LOBPCG (Alg. lobpcg_block), {n_iter} + {n_iter} iterations (restarted), ensemble "
                   f"generator seeds 4000-4001 with L 8-10, D 4-6, k 3-5; shifted frame (harmonic ZPE removed)",
           "n_iter": n_iter, "members": []}
    for mb in members:
        m = mb["model"]
        tree = wl.binary_tree(m.dims) if mb["kind"] == "c4-binary" else wl.fork_tree(m.dims, 4, 1)
        W = ttno.build_ttno(tree, m)
        bonds = wl.bond_dims(tree, mb["D"])
        x0 = wl.initial_block(tree, bonds, m.omega, m.dims, mb["k"], mb["seed"] + 17)
        runs = []
        xs = x0
        for _ in range(2):
            lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in xs])
            shift = float(np.min(lam0)) - 837.0
            xs, lam = solvers.lobpcg(tree, W, xs, solvers.LobpcgOptions(n_iter=n_iter, shift=shift))
            runs.append(list(map(float, lam)))
        out["members"].append({"seed": mb["seed"], "kind": mb["kind"], "L": mb["L"], "D": mb["D"], "k": mb["k"],
                               "zpe": m.zpe_harmonic, "lam_after_run": runs})
        print("member", mb["seed"], mb["kind"], mb["L"], mb["D"], mb["k"], "done", flush=True)
    return out


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c1_grow", "c3_cluster", "topologies", "e1", "c4_members"]
    if "c1" in which:
        res = c1_runs()
        with open(os.path.join(HERE, "c1_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote c1_oracle_runs.json")
    if "c1_grow" in which:
        res = c1_grow_runs()
        with open(os.path.join(HERE, "c1_grow_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote c1_grow_oracle_runs.json")
    if "c3_cluster" in which:
        res = c3_cluster_runs()
        with open(os.path.join(HERE, "c3s7_cluster_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote c3s7_cluster_oracle_runs.json")
    if "topologies" in which:
        res = topology_runs()
        with open(os.path.join(HERE, "topology_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote topology_oracle_runs.json")
    if "c4_members" in which:
        res = c4_member_runs()
        with open(os.path.join(HERE, "c4_member_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote c4_member_oracle_runs.json")
    if "e1" in which:
        res = e1_runs()
        with open(os.path.join(HERE, "e1_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote e1_oracle_runs.json")
