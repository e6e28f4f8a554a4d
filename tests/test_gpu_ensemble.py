"""The ensemble driver (one library context and stream per member, a host
thread pool, HIP-graph replay of the sweeps after their first runs, tiles
chosen by the autotuner) against stored oracle runs on two small members of
the ensemble generator (tests/golden/c4_member_oracle_runs.json, written by
tests/golden/make_golden.py from the oracle alone): FP64, two runs of two
block-LOBPCG iterations each; the second run restarts from the first run's
states and replays the captured sweeps."""
import json
import os

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c4_member_oracle_runs.json")


def test_ensemble_members_match_oracle():
    from paper_2512_15875_amd import ttn
    from paper_2512_15875_amd.ensemble import Ensemble, EnsembleOpts

    ttn.lib()
    gold = json.load(open(GOLD))
    members = wl.ensemble_members(2, seed0=4000, D_range=(4, 6), k_range=(3, 5), L_range=(8, 10))
    for mb, g in zip(members, gold["members"]):
        assert (mb["seed"], mb["kind"], mb["L"], mb["D"], mb["k"]) == (g["seed"], g["kind"], g["L"], g["D"], g["k"])
    opts = EnsembleOpts(low="fp64", iters_low=gold["n_iter"], iters_fp64=0, concurrent=True, threads=2, graphs=True,
                        autotune=True, workspace_bytes=256 << 20)
    ens = Ensemble(members, opts)
    try:
        for run in range(2):
            lams, _, flops = ens.run()
            assert flops > 0
            for lam, g in zip(lams, gold["members"]):
                ref = np.sort(np.array(g["lam_after_run"][run]) + g["zpe"])
                err = np.max(np.abs(lam - ref))
                assert err < 1e-4, (run, g["seed"], err)
    finally:
        ens.close()
