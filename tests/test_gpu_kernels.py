"""Kernel parity: the HIP path (through the C ABI) against the FP64 oracle on
identical inputs.  Norm-wise relative error gates: FP64 1e-12, FP32 1e-5,
BF16-in/FP32-accumulate 3e-2."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import ttn as ottn
from tests.gpu_util import TOL, env_setup as _env_setup, heff_setup as _setup, node_case, rel_err, to_dev

pytestmark = pytest.mark.gpu

T = None


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ttn.lib()
    return ttn


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0, workspace_bytes=2 << 30)


# (kappa, d, Db, M, Da, k): node classes of the workloads plus ragged shapes
CASES = [
    (1, 8, [8], [3], [8], 7),                              # binary-tree leaf
    (2, 6, [8, 8], [5, 4], [8, 8], 10),                    # MPS middle site
    (2, 9, [12, 9], [9, 5], [12, 9], 5),                   # fork chain node
    (3, 1, [12, 11, 10], [7, 13, 5], [12, 11, 10], 4),     # auxiliary branching node
    (3, 3, [17, 23, 5], [7, 3, 11], [17, 23, 5], 3),       # ragged, several tiles
    (3, 1, [24, 24, 24], [21, 14, 14], [24, 24, 24], 2),   # binary tree level-2 shape
    (2, 1, [24, 24], [63, 63], [24, 24], 3),               # binary-tree root shape
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dt", [0, 1, 2, 3])
def test_heff_apply_matches_oracle(api, ctx, case, dt):
    kappa, d, Db, M, Da, k = case
    tree, W, X, E, gt, gW, envs, tdt = _setup(api, ctx, kappa, d, Db, M, Da, k, 100 + kappa, dt)
    shift = np.linspace(-3.0, 5.0, k)
    alpha = np.linspace(0.5, 1.5, k)
    gX = to_dev(X, tdt)
    gY = torch.zeros((k,) + tuple(Db) + (d,), dtype=tdt, device="cuda")
    api.heff_apply_block(ctx, gt, gW, envs, 1, k, gX, gY, shift=to_dev(shift), alpha=to_dev(alpha),
                         flags=api.HEFF_APPLY, compute=dt)
    ctx.sync()
    Y = gY.double().cpu().numpy()
    for j in range(k):
        ein = {c: E[c][j] for c in tree.neighbours(1)}
        ref = alpha[j] * ottn.heff_apply(tree, 1, W, X[j], ein, shift[j]) if Db == Da else None
        if ref is None:
            ref = alpha[j] * ottn.heff_apply(tree, 1, W, X[j], ein, 0.0)
        assert rel_err(Y[j], ref) < TOL[dt], (case, dt, j)


@pytest.mark.parametrize("tile", [10, 11, 12, 13, 14, 15, 16])
@pytest.mark.parametrize("dt", [1, 3])
def test_unit_k_tiles_match_oracle(api, tile, dt, monkeypatch):
    """Every tile of the unit-stride-k kernel, forced at planning time (fresh
    context per tile), on an H_eff at a three-leg node without a physical leg,
    FP32 storage and FP64 storage with FP32 arithmetic: M and N ragged for
    every tile, contractions with a K tail (K % 32 != 0), against the oracle;
    the profile must name the kernel (and its FP64-storage instance)."""
    monkeypatch.setenv("TTN_FORCE_TILE", str(tile))
    ctx = api.Context(0, workspace_bytes=1 << 28)
    Db = Da = [15, 14, 13]
    M = [20, 12, 10]
    k = 3
    tree, W, X, E, gt, gW, envs, tdt = _setup(api, ctx, 3, 1, Db, M, Da, k, 91, dt)
    shift = np.linspace(-1.0, 2.0, k)
    gX = to_dev(X, tdt)
    gY = torch.zeros((k,) + tuple(Db) + (1,), dtype=tdt, device="cuda")
    api.profile(ctx, True)
    api.heff_apply_block(ctx, gt, gW, envs, 1, k, gX, gY, shift=to_dev(shift), compute=dt)
    rep = api.profile_report(ctx)
    api.profile(ctx, False)
    ctx.sync()
    kernels = {r[2] for r in rep}
    tn = [kn for kn in kernels if kn.startswith("ogemm_tn_kernel")]
    assert tn, kernels
    assert all(kn.endswith(", double>") == (dt == 3) for kn in tn), tn
    Y = gY.double().cpu().numpy()
    for j in range(k):
        ein = {c: E[c][j] for c in tree.neighbours(1)}
        ref = ottn.heff_apply(tree, 1, W, X[j], ein, shift[j])
        assert rel_err(Y[j], ref) < TOL[dt], (tile, dt, j)
    ctx.close()


@pytest.mark.parametrize("case", CASES[:5])
def test_heff_identity_operator_and_accumulate(api, ctx, case):
    kappa, d, Db, M, Da, k = case
    Da = [x + 1 if i == 0 else x for i, x in enumerate(Da)]  # bra != ket bonds (fitting RHS)
    tree, W, X, E, gt, gW, envs, tdt = _setup(api, ctx, kappa, d, Db, M, Da, k, 7 + kappa, api.F64, op=False)
    gX = to_dev(X)
    base = np.random.default_rng(1).normal(size=(k,) + tuple(Db) + (d,))
    gY = to_dev(base)
    alpha = np.linspace(-1.0, 2.0, k)
    api.heff_apply_block(ctx, gt, None, envs, 1, k, gX, gY, alpha=to_dev(alpha),
                         flags=api.HEFF_NO_SHIFT | api.HEFF_ACCUM, compute=api.F64)
    ctx.sync()
    Y = gY.cpu().numpy()
    for j in range(k):
        ein = {c: E[c][j] for c in tree.neighbours(1)}
        ref = base[j] + alpha[j] * ottn.heff_apply(tree, 1, None, X[j], ein)
        assert rel_err(Y[j], ref) < 1e-12


@pytest.mark.parametrize("dims", [[24, 24, 24], [12, 11, 10], [24, 8, 8]])
@pytest.mark.parametrize("dt", [1, 2])
@pytest.mark.parametrize("fused", [True, False])
def test_identity_heff_rows_fp32(api, ctx, dims, dt, fused, monkeypatch):
    """Identity-operator H_eff products of the fitting form (environment slot =
    item, X rows through a table, plain output) at three-leg nodes without a
    physical leg, in FP32 / BF16 compute against the oracle: the fused kernel
    and the staged path (switched by TTN_FUSED_IENV), checked in the profile."""
    monkeypatch.setenv("TTN_FUSED_IENV", "1" if fused else "0")
    n, kx = 7, 3
    tree, W, X, E, gt, gW, envs, tdt = _setup(api, ctx, 3, 1, dims, [1, 1, 1], dims, n, 61, dt, op=False)
    rng = np.random.default_rng(62)
    Xs = rng.normal(size=(kx,) + tuple(dims) + (1,))
    ids = np.array([2, 0, 1, 1, 0, 2, 2], dtype=np.int32)
    gY = torch.zeros((n,) + tuple(dims) + (1,), dtype=tdt, device="cuda")
    api.profile(ctx, True)
    api.heff_apply_block(ctx, gt, None, envs, 1, n, to_dev(Xs, tdt), gY,
                         x_ids=torch.from_numpy(ids).cuda(), flags=api.HEFF_NO_SHIFT, compute=dt)
    ctx.sync()
    kernels = {r[2] for r in api.profile_report(ctx)}
    api.profile(ctx, False)
    assert ("iheff3_kernel" in kernels) == fused, kernels
    Y = gY.double().cpu().numpy()
    for j in range(n):
        ein = {c: E[c][j] for c in tree.neighbours(1)}
        ref = ottn.heff_apply(tree, 1, None, Xs[ids[j]], ein)
        assert rel_err(Y[j], ref) < TOL[dt], (dims, dt, fused, j)


# (d, Db, M, Da, k): binary-tree leaf, fork chain tail, ragged, bra != ket bonds
LEAF_CASES = [(8, 8, 3, 8, 7), (14, 14, 5, 14, 4), (6, 5, 4, 5, 3), (9, 12, 7, 10, 5)]


@pytest.mark.parametrize("case", LEAF_CASES)
@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("fused", [True, False])
def test_leaf_heff_fused_and_staged(api, ctx, case, dt, fused, monkeypatch):
    """Operator H_eff products at a node with one virtual leg and a physical
    leg (tree leaves, MPS ends): the fused kernel and the staged path (switched
    by TTN_FUSED_LEAF, checked in the profile) against the oracle, with
    environment-slot and X-row tables, per-item scale, shift (square bonds)
    and accumulation into Y."""
    monkeypatch.setenv("TTN_FUSED_LEAF", "1" if fused else "0")
    d, Db, M, Da, k = case
    n_slots = k + 2
    tree, W, X, E = node_case(1, d, [Db], [M], [Da], k, 70 + d, op=True, n_slots=n_slots)
    _, _, _, _, gt, gW, envs, tdt = _setup(api, ctx, 1, d, [Db], [M], [Da], n_slots, 70 + d, dt)
    for c in tree.neighbours(1):
        envs.get(c, 1).copy_(to_dev(E[c], tdt))
    gW.W[1].copy_(to_dev(W, tdt))
    pair = np.array([(2 * j + 1) % n_slots for j in range(k)], dtype=np.int32)
    xid = np.array([k - 1 - j for j in range(k)], dtype=np.int32)
    base = np.random.default_rng(71).normal(size=(k, Db, d))
    gY = to_dev(base, tdt)
    square = Db == Da
    shift = np.linspace(-2.0, 3.0, k)
    alpha = np.linspace(0.5, 1.5, k)
    flags = api.HEFF_ACCUM | (0 if square else api.HEFF_NO_SHIFT)
    api.profile(ctx, True)
    api.heff_apply_block(ctx, gt, gW, envs, 1, k, to_dev(X, tdt), gY, pair_ids=torch.from_numpy(pair).cuda(),
                         x_ids=torch.from_numpy(xid).cuda(), shift=to_dev(shift) if square else None,
                         alpha=to_dev(alpha), flags=flags, compute=dt)
    ctx.sync()
    kernels = {r[2] for r in api.profile_report(ctx)}
    api.profile(ctx, False)
    assert ("leaf_heff_kernel" in kernels) == fused, kernels
    Y = gY.double().cpu().numpy()
    for j in range(k):
        ein = {c: E[c][pair[j]] for c in tree.neighbours(1)}
        ref = base[j] + alpha[j] * ottn.heff_apply(tree, 1, W, X[xid[j]], ein, shift[j] if square else 0.0)
        assert rel_err(Y[j], ref) < TOL[dt], (case, dt, fused, j)


@pytest.mark.parametrize("case", CASES[:6])
def test_heff_pair_and_row_indirection(api, ctx, case):
    kappa, d, Db, M, Da, k = case
    n_slots = k + 3
    tree, W, X, E = node_case(kappa, d, Db, M, Da, k, 55, op=True, n_slots=n_slots)
    # reuse _setup for handles, then overwrite the envs with n_slots slots
    tree2, W2, X2, E2, gt, gW, envs, tdt = _setup(api, ctx, kappa, d, Db, M, Da, n_slots, 55, api.F64)
    for c in tree.neighbours(1):
        envs.get(c, 1).copy_(to_dev(E[c]))
    gW.W[1].copy_(to_dev(W))
    pair = np.array([(3 * j + 1) % n_slots for j in range(k)], dtype=np.int32)
    xid = np.array([(k - 1 - j) for j in range(k)], dtype=np.int32)
    gY = torch.zeros((k,) + tuple(Db) + (d,), dtype=torch.float64, device="cuda")
    api.heff_apply_block(ctx, gt, gW, envs, 1, k, to_dev(X), gY, pair_ids=torch.from_numpy(pair).cuda(),
                         x_ids=torch.from_numpy(xid).cuda(), flags=api.HEFF_NO_SHIFT, compute=api.F64)
    ctx.sync()
    Y = gY.cpu().numpy()
    for j in range(k):
        ein = {c: E[c][pair[j]] for c in tree.neighbours(1)}
        ref = ottn.heff_apply(tree, 1, W, X[xid[j]], ein)
        assert rel_err(Y[j], ref) < 1e-12


@pytest.mark.parametrize("case", CASES)
def test_heff_diag_matches_oracle(api, ctx, case):
    kappa, d, Db, M, Da, k = case
    tree, W, X, E, gt, gW, envs, tdt = _setup(api, ctx, kappa, d, Db, M, Db, k, 31, api.F64)
    shift = np.linspace(1.0, 2.0, k)
    gY = torch.zeros((k,) + tuple(Db) + (d,), dtype=torch.float64, device="cuda")
    api.heff_apply_block(ctx, gt, gW, envs, 1, k, None, gY, shift=to_dev(shift), flags=api.HEFF_DIAG,
                         compute=api.F64)
    ctx.sync()
    Y = gY.cpu().numpy()
    for j in range(k):
        ein = {c: E[c][j] for c in tree.neighbours(1)}
        ref = ottn.heff_diag(tree, 1, W, ein, shift[j])
        assert rel_err(Y[j], ref) < 1e-12


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("dt", [0, 1, 2])
def test_env_update_matches_oracle(api, ctx, case, dt):
    kappa, d, Db, M, Da, _ = case
    Da = [x + (1 if i == kappa - 1 else 0) for i, x in enumerate(Da)]
    tree, gt, bra, ket, A_b, A_k, W, gW, envs, E, pairs, pb, pk, tdt = _env_setup(
        api, ctx, kappa, d, Db, M, Da, 2, 3, 200 + kappa, dt)
    nb = tree.neighbours(1)
    for v in nb:
        api.ttno_env_update(ctx, gt, gW, bra, ket, pb, pk, 1, v, envs, dt)
        ctx.sync()
        got = envs.get(1, v).double().cpu().numpy()
        for p, (i, j) in enumerate(pairs):
            ein = {c: E[c][p] for c in nb if c != v}
            ref = ottn.env_update(tree, 1, v, A_b[i], W, A_k[j], ein)
            assert rel_err(got[p], ref) < TOL[dt], (case, dt, v, p)


@pytest.mark.parametrize("dt", [0, 1])
def test_env_update_long_contraction(api, ctx, dt):
    """Operator environments at a node with three 40-dimensional bonds, where
    a stage contracts two bonds at once (K = 1600, beyond the 1536 entries up
    to which the GEMM stages its k-offset tables in LDS): the global-table
    main loop, checked in the profile, against the oracle."""
    kappa, d, Db, M, Da = 3, 1, [40, 40, 40], [3, 4, 2], [40, 40, 40]
    tree, gt, bra, ket, A_b, A_k, W, gW, envs, E, pairs, pb, pk, tdt = _env_setup(
        api, ctx, kappa, d, Db, M, Da, 2, 2, 207, dt)
    nb = tree.neighbours(1)
    api.profile(ctx, True)
    for v in nb:
        api.ttno_env_update(ctx, gt, gW, bra, ket, pb, pk, 1, v, envs, dt)
        ctx.sync()
        got = envs.get(1, v).double().cpu().numpy()
        for p, (i, j) in enumerate(pairs):
            ein = {c: E[c][p] for c in nb if c != v}
            ref = ottn.env_update(tree, 1, v, A_b[i], W, A_k[j], ein)
            assert rel_err(got[p], ref) < TOL[dt], (dt, v, p)
    ks = [r[8] for r in api.profile_report(ctx)]
    api.profile(ctx, False)
    assert max(ks) > 1536, ks


@pytest.mark.parametrize("case", CASES[:5])
def test_env_update_identity_and_closure(api, ctx, case):
    kappa, d, Db, M, Da, _ = case
    for op in (False, True):
        tree, gt, bra, ket, A_b, A_k, W, gW, envs, E, pairs, pb, pk, tdt = _env_setup(
            api, ctx, kappa, d, Db, M, Da, 3, 2, 300 + kappa, api.F64, op=op)
        nb = tree.neighbours(1)
        v = nb[-1]
        api.ttno_env_update(ctx, gt, gW, bra, ket, pb, pk, 1, v, envs, api.F64)
        out = torch.zeros(len(pairs), dtype=torch.float64, device="cuda")
        api.ttno_env_close(ctx, gt, gW, bra, ket, pb, pk, 1, envs, out, api.F64)
        ctx.sync()
        got = envs.get(1, v).cpu().numpy()
        cl = out.cpu().numpy()
        for p, (i, j) in enumerate(pairs):
            ein = {c: E[c][p] for c in nb if c != v}
            ref = ottn.env_update(tree, 1, v, A_b[i], W, A_k[j], ein)
            assert rel_err(got[p], ref) < 1e-12
            ref_c = ottn.closure(tree, 1, A_b[i], W, A_k[j], {c: E[c][p] for c in nb})
            assert abs(cl[p] - ref_c) <= 1e-12 * max(1.0, abs(ref_c)) * 10


def test_rejects_bad_arguments(api, ctx):
    kappa, d, Db, M, Da, k = CASES[1]
    tree, W, X, E, gt, gW, envs, tdt = _setup(api, ctx, kappa, d, Db, M, Da, k, 1, api.F64)
    gY = torch.zeros((k,) + tuple(Db) + (d,), dtype=torch.float64, device="cuda")
    with pytest.raises(api.TTNError):  # wrong compute dtype for F64 tensors
        api.heff_apply_block(ctx, gt, gW, envs, 1, k, to_dev(X), gY, compute=api.F32)
    with pytest.raises(api.TTNError):  # bad node
        api.heff_apply_block(ctx, gt, gW, envs, 7, k, to_dev(X), gY, compute=api.F64)
    with pytest.raises(api.TTNError):  # k beyond the env slots
        api.heff_apply_block(ctx, gt, gW, envs, 1, k + 1, to_dev(X), gY, compute=api.F64)
    # k = 0 is a no-op
    api.heff_apply_block(ctx, gt, gW, envs, 1, 0, to_dev(X), gY, compute=api.F64)


# the binary-tree node above two leaves (24 to the parent, 8 to each leaf)
IENV_EXTRA = [(3, 1, [24, 8, 8], [1, 1, 1], [24, 8, 8], 2)]


@pytest.mark.parametrize("case", CASES + IENV_EXTRA)
@pytest.mark.parametrize("dt", [1, 2])
@pytest.mark.parametrize("fused", [True, False])
def test_identity_env_update_fp32_paths(api, ctx, case, dt, fused, monkeypatch):
    """Identity-operator environment updates (the overlap environments of the
    Gram step and of fitting) in FP32 / BF16 compute, every direction, against
    the oracle.  Three-leg nodes without a physical leg take the fused kernel
    (intermediates in LDS) unless it is switched off; staged, the binary-tree
    node shape goes through the split-K skinny kernel (both checked in the
    stage profile)."""
    monkeypatch.setenv("TTN_FUSED_IENV", "1" if fused else "0")
    kappa, d, Db, M, Da, _ = case
    tree, gt, bra, ket, A_b, A_k, W, gW, envs, E, pairs, pb, pk, tdt = _env_setup(
        api, ctx, kappa, d, Db, M, Db, 3, 4, 400 + kappa, dt, op=False)
    nb = tree.neighbours(1)
    api.profile(ctx, True)
    for v in nb:
        api.ttno_env_update(ctx, gt, None, bra, ket, pb, pk, 1, v, envs, dt)
        ctx.sync()
        got = envs.get(1, v).double().cpu().numpy()
        for p, (i, j) in enumerate(pairs):
            ein = {c: E[c][p] for c in nb if c != v}
            ref = ottn.env_update(tree, 1, v, A_b[i], None, A_k[j], ein)
            assert rel_err(got[p], ref) < TOL[dt], (case, dt, v, p)
    kernels = {r[2] for r in api.profile_report(ctx)}
    api.profile(ctx, False)
    if kappa == 3 and d == 1:
        assert ("ienv3_kernel" in kernels) == fused, kernels
    if Db == [24, 24, 24] and not fused:  # the binary-tree node: a 24 x 24 x 576 closing stage
        assert "ogemm_splitk_kernel" in kernels, kernels
