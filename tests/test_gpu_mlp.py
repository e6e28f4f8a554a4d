"""The learned local preconditioner on the GPU against the oracle
(oracle.mlp): network forward, backward, loss and Adam through the C ABI in
FP32 and BF16 matrix-core arithmetic, tile features and targets, sweep
harvesting, and the DIAG / LEARNED local maps of an ALS sweep."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import mlp as omlp
from oracle import solvers as osol
from oracle import ttn as ottn
from oracle import ttno as ottno
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu

# norm-wise relative tolerances: FP32 operands with FP32 accumulation, and
# bfloat16-rounded operands (8-bit significand) with FP32 accumulation
TOL = {"f32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    ttn.lib()
    return ttn


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0, workspace_bytes=1 << 30)


def _params(seed):
    rng = np.random.default_rng(seed)
    p = omlp.init_params(seed)
    W1, b1, W2, b2, W3, b3 = omlp.unpack(p)
    W3 *= 10.0
    b1 += rng.normal(scale=0.3, size=b1.shape)
    b2 += rng.normal(scale=0.3, size=b2.shape)
    b3 += rng.normal(scale=0.3, size=b3.shape)
    return p.astype(np.float32).astype(np.float64)  # the values the GPU holds


def _f32(a):
    return to_dev(a, torch.float32)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("n", [1, 1000])
def test_forward_backward_match_oracle(api, ctx, prec, n):
    comp = api.F32 if prec == "f32" else api.BF16
    rng = np.random.default_rng(n)
    p = _params(21)
    X = rng.normal(size=(n, 128)).astype(np.float32).astype(np.float64)
    dY = rng.normal(size=(n, 64)).astype(np.float32).astype(np.float64)
    Y_ref, cache = omlp.forward(p, X)
    g_ref = omlp.backward(p, cache, dY)
    pd, Xd, dYd = _f32(p), _f32(X), _f32(dY)
    Yd = torch.empty(n, 64, dtype=torch.float32, device="cuda")
    acts = torch.empty(4, n, 256, dtype=torch.float32, device="cuda")
    grads = torch.empty(omlp.n_params(), dtype=torch.float32, device="cuda")
    api.mlp_forward(ctx, pd, Xd, Yd, acts, comp)
    api.mlp_backward(ctx, pd, Xd, acts, dYd, grads, comp)
    ctx.sync()
    assert rel_err(Yd.cpu().numpy(), Y_ref) < TOL[prec]
    assert rel_err(acts[1].cpu().numpy(), cache["h1"]) < TOL[prec]
    g = grads.cpu().numpy()
    bounds = np.cumsum([0] + [s for i, o in omlp.SIZES for s in (i * o, o)])
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        assert rel_err(g[lo:hi], g_ref[lo:hi]) < TOL[prec], (lo, hi)
    # forward without kept activations gives the same output
    Y2 = torch.empty_like(Yd)
    api.mlp_forward(ctx, pd, Xd, Y2, None, comp)
    ctx.sync()
    assert torch.equal(Y2, Yd)


def test_loss_and_adam_match_oracle(api, ctx):
    rng = np.random.default_rng(4)
    n = 333
    Y = rng.normal(size=(n, 64)).astype(np.float32).astype(np.float64)
    T = rng.normal(size=(n, 64)).astype(np.float32).astype(np.float64)
    loss_ref, dY_ref = omlp.mse(Y, T)
    dY = torch.empty(n, 64, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.mlp_loss(ctx, _f32(Y), _f32(T), dY, loss)
    ctx.sync()
    assert abs(loss.item() - loss_ref) <= 1e-12 * loss_ref
    assert rel_err(dY.cpu().numpy(), dY_ref) < 1e-6
    # three Adam steps with changing gradients
    P = omlp.n_params()
    p = rng.normal(size=P).astype(np.float32).astype(np.float64)
    m = np.zeros(P)
    v = np.zeros(P)
    pd, md, vd = _f32(p), torch.zeros(P, dtype=torch.float32, device="cuda"), torch.zeros(
        P, dtype=torch.float32, device="cuda")
    for step in (1, 2, 3):
        g = rng.normal(size=P).astype(np.float32).astype(np.float64)
        p, m, v = omlp.adam_step(p, m, v, g, 1e-3, step)
        api.mlp_adam(ctx, pd, md, vd, _f32(g), 1e-3, step)
    ctx.sync()
    # parameters move by O(lr) per step: compare the update, not the values
    p0 = pd.cpu().numpy()
    assert np.max(np.abs(p0 - p)) < 1e-6


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_features_and_targets_match_oracle(api, ctx, dt):
    tdt = torch.float64 if dt == "f64" else torch.float32
    rng = np.random.default_rng(9)
    k, n = 3, 130
    b = rng.normal(size=(k, n))
    d = rng.uniform(0.5, 4.0, size=(k, n)) * rng.choice([-1, 1], size=(k, n))
    y = rng.normal(size=(k, n))
    if dt == "f32":
        b, d, y = (a.astype(np.float32).astype(np.float64) for a in (b, d, y))
    nt = -(-n // 64)
    X = torch.empty(k * nt, 128, dtype=torch.float32, device="cuda")
    T = torch.empty(k * nt, 64, dtype=torch.float32, device="cuda")
    sc = torch.empty(k, 2, dtype=torch.float64, device="cuda")
    api.precond_features(ctx, to_dev(b, tdt), to_dev(d, tdt), sc, X)
    api.precond_targets(ctx, to_dev(y, tdt), to_dev(b, tdt), to_dev(d, tdt), sc, T)
    ctx.sync()
    for j in range(k):
        Xr, scr = omlp.features(b[j], d[j])
        assert np.allclose(sc[j].cpu().numpy(), scr, rtol=1e-12, atol=0)
        assert rel_err(X[j * nt:(j + 1) * nt].cpu().numpy(), Xr) < 1e-7
        assert rel_err(T[j * nt:(j + 1) * nt].cpu().numpy(), omlp.targets(y[j], b[j], d[j], scr)) < 1e-7


def test_training_reduces_loss(api, ctx):
    """Adam on the GPU kernels fits a smooth synthetic map (property: the
    loss falls by an order of magnitude)."""
    rng = np.random.default_rng(12)
    n = 2048
    X = rng.normal(size=(n, 128))
    Tt = np.tanh(X[:, :64] * 0.5) * X[:, 64:] * 0.3
    p = omlp.init_params(5)
    pd = _f32(p)
    Xd, Td = _f32(X), _f32(Tt)
    P = omlp.n_params()
    md = torch.zeros(P, dtype=torch.float32, device="cuda")
    vd = torch.zeros_like(md)
    Yd = torch.empty(n, 64, dtype=torch.float32, device="cuda")
    acts = torch.empty(4, n, 256, dtype=torch.float32, device="cuda")
    dY = torch.empty_like(Yd)
    g = torch.empty(P, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    for step in range(1, 301):
        api.mlp_forward(ctx, pd, Xd, Yd, acts, api.BF16)
        api.mlp_loss(ctx, Yd, Td, dY, loss)
        api.mlp_backward(ctx, pd, Xd, acts, dY, g, api.BF16)
        api.mlp_adam(ctx, pd, md, vd, g, 2e-3, step)
        if step in (1, 300):
            ctx.sync()
            hist.append(loss.item())
    assert np.isfinite(hist[-1]) and hist[-1] < 0.1 * hist[0], hist


# ---------------------------------------------------------------- sweeps


def _setup(api, ctx, k, D=6, seed=5):
    m = wl.quartic_force_field(8, 21, 20, 30)
    tree = wl.fork_tree(m.dims, 4, 1)
    W = ottno.build_ttno(tree, m)
    M = ottno.ttno_bonds(tree, W)
    bonds = wl.bond_dims(tree, D)
    gt = api.Tree(tree.parent, tree.phys)
    op = api.TTNO(ctx, gt, [to_dev(w) for w in W], [max(1, x) for x in M], api.F64)
    phi = wl.random_block(tree, bonds, k, seed)
    return tree, W, bonds, gt, op, phi


def _upload(api, ctx, gt, tree, bonds, states, k):
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], api.F64)
    for u in range(tree.n):
        blk.t[u].copy_(to_dev(np.stack([states[j][u] for j in range(k)])))
    return blk


def test_harvest_matches_oracle(api, ctx):
    k = 2
    tree, W, bonds, gt, op, phi = _setup(api, ctx, k)
    y0 = [ottn.canonicalize(tree, p, tree.root) for p in wl.random_block(tree, bonds, k, 6)]
    shifts = [-300.0, -50.0]
    Y = _upload(api, ctx, gt, tree, bonds, y0, k)
    P = _upload(api, ctx, gt, tree, bonds, phi, k)
    sw = api.Sweep(ctx, gt, op, Y, [(None, P, [0, 1], [0, 1], None)], shift=to_dev(np.array(shifts)),
                   compute=api.F64)
    r = tree.root
    sw.init(r)
    n = int(np.prod(y0[0][r].shape))
    nt = -(-n // 64)
    X = torch.empty(k * nt, 128, dtype=torch.float32, device="cuda")
    T = torch.empty(k * nt, 64, dtype=torch.float32, device="cuda")
    sc = torch.empty(k, 2, dtype=torch.float64, device="cuda")
    sw.harvest(r, X, T, sc)
    ctx.sync()
    for j in range(k):
        H = ottn.all_envs_toward(tree, r, y0[j], W, y0[j])
        R = ottn.all_envs_toward(tree, r, y0[j], None, phi[j])
        inc = lambda E: {c: E[(c, r)] for c in ottn.nbrs(tree, r)}
        b = ottn.heff_apply(tree, r, None, phi[j][r], inc(R)).ravel()
        d = ottn.heff_diag(tree, r, W[r], inc(H), shifts[j]).ravel()
        Xr, scr = omlp.features(b, d)
        assert np.allclose(sc[j].cpu().numpy(), scr, rtol=1e-10, atol=0)
        assert rel_err(X[j * nt:(j + 1) * nt].cpu().numpy(), Xr) < 1e-7
        assert rel_err(T[j * nt:(j + 1) * nt].cpu().numpy(), omlp.targets(y0[j][r].ravel(), b, d, scr)) < 1e-7


@pytest.mark.parametrize("local", ["diag", "learned"])
def test_als_local_maps_match_oracle(api, ctx, local):
    k = 3
    tree, W, bonds, gt, op, phi = _setup(api, ctx, k)
    y0 = [ottn.canonicalize(tree, p, tree.root) for p in phi]
    shifts = [-400.0, -150.0, -900.0]
    p = _params(33)
    Y = _upload(api, ctx, gt, tree, bonds, y0, k)
    P = _upload(api, ctx, gt, tree, bonds, phi, k)
    sw = api.Sweep(ctx, gt, op, Y, [(None, P, list(range(k)), list(range(k)), None)],
                   shift=to_dev(np.array(shifts)), compute=api.F64)
    sw.init(tree.root)
    if local == "diag":
        api.run_sweep(sw, gt, api.SOLVE_DIAG)
    else:
        api.run_sweep(sw, gt, api.SOLVE_LEARNED, mlp=_f32(p), mlp_compute=api.F32)
    ctx.sync()
    tol = 1e-10 if local == "diag" else 1e-4
    for j in range(k):
        ref = osol.als_solve(tree, W, shifts[j], phi[j], phi[j], sweeps=1, maxiter=0, rtol=0.0,
                             local="diag" if local == "diag" else ("learned", p))
        for u in range(tree.n):
            assert rel_err(Y.t[u][j].cpu().numpy(), ref[u]) < tol, (j, u)


@pytest.mark.parametrize("warm", ["diag", "learned"])
def test_als_corrected_minres_start_matches_oracle(api, ctx, warm):
    """MINRES local solves from a DIAG- or learned-corrected start (fixed
    iteration count) against the oracle's ALS with the same start."""
    k = 3
    tree, W, bonds, gt, op, phi = _setup(api, ctx, k)
    y0 = [ottn.canonicalize(tree, p, tree.root) for p in phi]
    shifts = [-400.0, -150.0, -900.0]
    p = _params(34)
    Y = _upload(api, ctx, gt, tree, bonds, y0, k)
    P = _upload(api, ctx, gt, tree, bonds, phi, k)
    sw = api.Sweep(ctx, gt, op, Y, [(None, P, list(range(k)), list(range(k)), None)],
                   shift=to_dev(np.array(shifts)), compute=api.F64)
    w = api.WARM_DIAG if warm == "diag" else api.WARM_LEARNED
    kw = dict(maxiter=4, rtol=0.0, mlp=_f32(p), mlp_compute=api.F32, warm=w)
    sw.run(api.SOLVE_MINRES, 1, init=True, **kw)
    ctx.sync()
    tol = 1e-8 if warm == "diag" else 1e-4
    for j in range(k):
        ref = osol.als_solve(tree, W, shifts[j], phi[j], phi[j], sweeps=1, maxiter=4, rtol=0.0,
                             local="minres+diag" if warm == "diag" else ("minres+learned", p))
        for u in range(tree.n):
            assert rel_err(Y.t[u][j].cpu().numpy(), ref[u]) < tol, (j, u)


def test_corrected_start_rejects_refinement(api, ctx):
    k = 2
    tree, W, bonds, gt, op, phi = _setup(api, ctx, k)
    y0 = [ottn.canonicalize(tree, p, tree.root) for p in phi]
    Y = _upload(api, ctx, gt, tree, bonds, y0, k)
    P = _upload(api, ctx, gt, tree, bonds, phi, k)
    sw = api.Sweep(ctx, gt, op, Y, [(None, P, [0, 1], [0, 1], None)], shift=to_dev(np.array([-300.0, -300.0])),
                   compute=api.F64)
    sw.init(tree.root)
    with pytest.raises(api.TTNError):
        sw.step(tree.root, -1, api.SOLVE_MINRES, maxiter=3, rtol=0.0, refine=2, warm=api.WARM_DIAG)
    with pytest.raises(api.TTNError):
        sw.step(tree.root, -1, api.SOLVE_MINRES, maxiter=3, rtol=0.0, warm=7)


def test_learned_step_never_worse_than_scaled_diag(api, ctx):
    """With corrupted (huge random) weights the combination falls back to the
    DIAG direction: the local residual is no larger than DIAG's at its best
    scale, node by node."""
    k = 2
    tree, W, bonds, gt, op, phi = _setup(api, ctx, k, seed=7)
    y0 = [ottn.canonicalize(tree, p, tree.root) for p in phi]
    shifts = [-500.0, -200.0]
    rng = np.random.default_rng(1)
    bad = _f32(rng.normal(scale=50.0, size=omlp.n_params()))
    Y = _upload(api, ctx, gt, tree, bonds, y0, k)
    P = _upload(api, ctx, gt, tree, bonds, phi, k)
    sw = api.Sweep(ctx, gt, op, Y, [(None, P, [0, 1], [0, 1], None)], shift=to_dev(np.array(shifts)),
                   compute=api.F64)
    r = tree.root
    sw.init(r)
    coef = torch.zeros(k, 2, dtype=torch.float64, device="cuda")
    sw.step(r, -1, api.SOLVE_LEARNED, mlp=bad, mlp_compute=api.BF16, learned_coef=coef)
    ctx.sync()
    for j in range(k):
        H = ottn.all_envs_toward(tree, r, y0[j], W, y0[j])
        R = ottn.all_envs_toward(tree, r, y0[j], None, phi[j])
        inc = lambda E: {c: E[(c, r)] for c in ottn.nbrs(tree, r)}
        b = ottn.heff_apply(tree, r, None, phi[j][r], inc(R))
        d = ottn.heff_diag(tree, r, W[r], inc(H), shifts[j])
        A = lambda v: ottn.heff_apply(tree, r, W[r], v, inc(H), shifts[j])
        yD = b / d
        Pd = A(yD).ravel()
        diag_best = np.linalg.norm((Pd @ b.ravel() / (Pd @ Pd)) * Pd - b.ravel())
        got = Y.t[r][j].cpu().numpy()
        res = np.linalg.norm((A(got) - b).ravel())
        assert np.isfinite(res) and res <= diag_best * (1 + 1e-9), (res, diag_best)
    assert torch.isfinite(coef).all()
