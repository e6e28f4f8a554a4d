"""Sweep executor, HIP-graph replay and the tile autotuner: graph replays
and autotuned launches must reproduce the eager, untuned results (replayed
several times with eager work and synchronisations between replays), and the
native Euler-tour executor must match the host-driven tour."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import ttno as ottno
from oracle import ttn as ottn
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    ttn.lib()
    return ttn


def _problem(api, ctx, k=3, D=6, seed=5):
    m = wl.quartic_force_field(8, 21, 20, 30)
    tree = wl.fork_tree(m.dims, 4, 1)
    W = ottno.build_ttno(tree, m)
    M = ottno.ttno_bonds(tree, W)
    bonds = wl.bond_dims(tree, D)
    gt = api.Tree(tree.parent, tree.phys)
    op = api.TTNO(ctx, gt, [to_dev(w) for w in W], [max(1, x) for x in M], api.F64)
    phi = wl.random_block(tree, bonds, k, seed)
    y0 = [ottn.canonicalize(tree, p, tree.root) for p in phi]

    def block(states):
        b = api.Block(ctx, gt, k, [max(1, x) for x in bonds], api.F64)
        for u in range(tree.n):
            b.t[u].copy_(to_dev(np.stack([states[j][u] for j in range(k)])))
        return b
    return tree, gt, op, phi, y0, block


def _snapshot(blk, n):
    return [blk.t[u].clone() for u in range(n)]


def _restore(blk, snap):
    for u, t in enumerate(snap):
        blk.t[u].copy_(t)


@pytest.mark.parametrize("mode", ["fit", "minres", "diag", "minres_diag_start"])
def test_graph_replays_match_eager(api, mode):
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = api.Context(0, workspace_bytes=1 << 28, stream=stream)
        k = 3
        tree, gt, op, phi, y0, block = _problem(api, ctx, k)
        Y, P = block(y0), block(phi)
        idx = list(range(k))
        if mode == "fit":
            coef = to_dev(np.array([0.5, -1.0, 2.0]))
            sw = api.Sweep(ctx, gt, None, Y, [(op, P, idx, idx, coef)], compute=api.F64)
            m, kw = api.SOLVE_FIT, {}
        else:
            sh = to_dev(np.array([-300.0, -100.0, -700.0]))
            sw = api.Sweep(ctx, gt, op, Y, [(None, P, idx, idx, None)], shift=sh, compute=api.F64)
            m, kw = {"minres": (api.SOLVE_MINRES, {"maxiter": 6}), "diag": (api.SOLVE_DIAG, {}),
                     "minres_diag_start": (api.SOLVE_MINRES, {"maxiter": 6, "warm": api.WARM_DIAG})}[mode]
        start = _snapshot(Y, tree.n)
        # eager reference
        sw.run(m, 2, init=True, graph=False, **kw)
        ref = _snapshot(Y, tree.n)
        # first graph call runs eagerly, second captures, later ones replay
        for rep in range(4):
            _restore(Y, start)
            sw.run(m, 2, init=True, graph=True, **kw)
            ctx.sync()
            for u in range(tree.n):
                assert torch.equal(Y.t[u], ref[u]), (rep, u)
            # unrelated eager work between replays
            x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
            (x * 2).sum().item()
        ctx.sync()


def test_native_tour_matches_host_tour(api):
    ctx = api.Context(0, workspace_bytes=1 << 28)
    k = 2
    tree, gt, op, phi, y0, block = _problem(api, ctx, k, seed=9)
    results = []
    for native in (True, False):
        Y, P = block(y0), block(phi)
        sh = to_dev(np.array([-400.0, -50.0]))
        sw = api.Sweep(ctx, gt, op, Y, [(None, P, [0, 1], [0, 1], None)], shift=sh, compute=api.F64)
        sw.init(tree.root)
        its = torch.zeros(k, dtype=torch.int32, device="cuda")
        if native:
            api.run_sweep(sw, gt, api.SOLVE_MINRES, 5, 0.0, iters=its)
        else:
            api.run_sweep(sw, gt, api.SOLVE_MINRES, 5, 0.0, collect=[])  # the host-driven tour
        ctx.sync()
        results.append(_snapshot(Y, tree.n))
    for u in range(tree.n):
        assert torch.equal(results[0][u], results[1][u]), u


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotuned_solver_matches_untuned(api, prec):
    from paper_2512_15875_amd.solver import LobpcgOpts, TTNEigensolver
    m = wl.make_config_model("c3")
    tree = wl.fork_tree(m.dims, 4, 1)
    bonds = wl.bond_dims(tree, 8)
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, 6, m.seed + 17)
    lams = []
    for tune in (False, True):
        ctx = api.Context(0, workspace_bytes=1 << 29)
        api.autotune(ctx, tune)
        s = TTNEigensolver(ctx, tree, m, D=8, k=6, precision=prec)
        s.load_block(x0)
        lams.append(s.lobpcg(LobpcgOpts(n_iter=2)))
        log = api.autotune(ctx, None)
        assert (len(log.splitlines()) > 10) == tune
        del s
        ctx.close()  # also destroys any sweep still alive on it
    # tile shapes change the order of the FP32 partial sums (the split-K kernel
    # sums four k-interleaved partials), so FP32 runs agree to FP32 rounding
    # amplified by two LOBPCG iterations: 5e-6 relative (about 0.05 cm^-1 at 1e4)
    tol = 1e-9 if prec == "fp64" else 5e-6 * np.max(np.abs(lams[0]))
    assert np.max(np.abs(lams[0] - lams[1])) < tol
