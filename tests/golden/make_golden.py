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


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "c3_cluster"]
    if "c1" in which:
        res = c1_runs()
        with open(os.path.join(HERE, "c1_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote c1_oracle_runs.json")
    if "c3_cluster" in which:
        res = c3_cluster_runs()
        with open(os.path.join(HERE, "c3s7_cluster_oracle_runs.json"), "w") as f:
            json.dump(res, f, indent=1)
        print("wrote c3s7_cluster_oracle_runs.json")
