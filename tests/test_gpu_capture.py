"""The boundary's capture contract: after the *_create calls nothing
allocates device memory, and a MINRES sweep with more than one convergence
segment (maxiter > 25) can be captured into a HIP graph and replayed; the
replays equal the eager run bit for bit and match the oracle's ALS."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import solvers as osol
from oracle import ttn as ottn
from oracle import ttno as ottno
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    ttn.lib()
    return ttn


def test_captured_minres_sweep_allocates_nothing(api):
    """An inverse-iteration-style ALS sweep (H - s_j) y_j = x_j, MINRES
    maxiter 60 and rtol 1e-10: eagerly, then captured once and replayed three
    times with eager work between the replays."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = api.Context(0, workspace_bytes=1 << 28, stream=stream)
        m = wl.quartic_force_field(8, 21, 20, 30)
        tree = wl.fork_tree(m.dims, 4, 1)
        W = ottno.build_ttno(tree, m)
        M = ottno.ttno_bonds(tree, W)
        bonds = wl.bond_dims(tree, 6)
        gt = api.Tree(tree.parent, tree.phys)
        op = api.TTNO(ctx, gt, [to_dev(w) for w in W], [max(1, x) for x in M], api.F64)
        k = 3
        phi = wl.random_block(tree, bonds, k, 41)
        y0 = [ottn.canonicalize(tree, p, tree.root) for p in phi]

        def block(states):
            b = api.Block(ctx, gt, k, [max(1, x) for x in bonds], api.F64)
            for u in range(tree.n):
                b.t[u].copy_(to_dev(np.stack([states[j][u] for j in range(k)])))
            return b

        Y, P = block(y0), block(phi)
        shifts = [-250.0, -120.0, -600.0]
        sw = api.Sweep(ctx, gt, op, Y, [(None, P, list(range(k)), list(range(k)), None)],
                       shift=to_dev(np.array(shifts)), compute=api.F64)
        iters = torch.zeros(k, dtype=torch.int32, device="cuda")
        start = [Y.t[u].clone() for u in range(tree.n)]
        sw.run(api.SOLVE_MINRES, 1, init=True, graph=False, maxiter=60, rtol=1e-10, iters=iters)
        ctx.sync()
        ref = [Y.t[u].clone() for u in range(tree.n)]
        n_alloc = api.alloc_count()
        for rep in range(4):  # eager (plans), capture + launch, replay, replay
            for u in range(tree.n):
                Y.t[u].copy_(start[u])
            sw.run(api.SOLVE_MINRES, 1, init=True, graph=True, maxiter=60, rtol=1e-10, iters=iters)
            ctx.sync()
            for u in range(tree.n):
                assert torch.equal(Y.t[u], ref[u]), (rep, u)
            x = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
            (x * 2).sum().item()
        assert api.alloc_count() == n_alloc
        ctx.sync()
        for j in range(k):
            oref = osol.als_solve(tree, W, shifts[j], phi[j], phi[j], sweeps=1, maxiter=60, rtol=1e-10)
            for u in range(tree.n):
                assert rel_err(Y.t[u][j].cpu().numpy(), oref[u]) < 1e-8, (j, u)


def test_solver_steps_allocate_nothing(api):
    """Once the solver's sweeps exist (the first inverse-iteration call creates
    its two) and the plans are built, further LOBPCG iterations, inverse
    iteration with clusters and the final Rayleigh-Ritz make no library
    allocation."""
    from paper_2512_15875_amd.solver import IIOpts, LobpcgOpts, TTNEigensolver
    ctx = api.Context(0, workspace_bytes=1 << 28)
    m = wl.make_config_model("c3", seed=7)
    tree = wl.fork_tree(m.dims, 4, 1)
    bonds = wl.bond_dims(tree, 8)
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, 12, m.seed + 17)
    s = TTNEigensolver(ctx, tree, m, D=8, k=12, precision="fp64")
    s.load_block(x0)
    s.lobpcg_start(LobpcgOpts(n_iter=5))
    for _ in range(3):  # the stored oracle run of this case holds two clusters of two states here
        s.lobpcg_step()
    s.inverse_iteration(IIOpts(n_iter=1, minres_maxiter=200))
    ctx.sync()
    assert s.cluster_rr_calls == 1
    n_alloc = api.alloc_count()
    s.lobpcg_step()
    s.inverse_iteration(IIOpts(n_iter=1, minres_maxiter=200))
    ctx.sync()
    assert s.cluster_rr_calls == 2
    assert api.alloc_count() == n_alloc
