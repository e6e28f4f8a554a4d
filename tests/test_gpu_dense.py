"""GPU Rayleigh-Ritz, QR gauge move and node norms against the oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import linalg as olin
from oracle import ttn as ottn
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    ttn.lib()
    return ttn


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0, workspace_bytes=1 << 30)


@pytest.mark.parametrize("m,nev", [(6, 3), (30, 10), (97, 20), (252, 84)])
def test_rayleigh_ritz_cholesky_matches_oracle(api, ctx, m, nev):
    rng = np.random.default_rng(m)
    batch = 3
    ld = m + 3
    H = np.zeros((batch, ld, ld))
    S = np.zeros((batch, ld, ld))
    ms = [m, max(1, m - 2), m]
    for b in range(batch):
        mm = ms[b]
        A = rng.normal(size=(mm, mm)) * 100
        B = rng.normal(size=(mm, mm))
        H[b, :mm, :mm] = A + A.T
        S[b, :mm, :mm] = B @ B.T / mm + np.eye(mm)
    ev, V, rank = api.rayleigh_ritz(ctx, to_dev(H), to_dev(S), ms, nev)
    ctx.sync()
    ev, V, rank = ev.cpu().numpy(), V.cpu().numpy(), rank.cpu().numpy()
    for b in range(batch):
        mm = ms[b]
        ne = min(nev, mm)
        lam, Vr, rk = olin.rayleigh_ritz(H[b, :mm, :mm], S[b, :mm, :mm], ne)
        assert rank[b] == rk == mm
        np.testing.assert_allclose(ev[b, :ne], lam, rtol=0, atol=1e-10 * np.abs(lam).max())
        # eigenvectors: unique up to sign for simple eigenvalues; same sign convention
        np.testing.assert_allclose(V[b, :mm, :ne], Vr, atol=1e-8)
        G = V[b, :mm, :ne].T @ S[b, :mm, :mm] @ V[b, :mm, :ne]
        np.testing.assert_allclose(G, np.eye(ne), atol=1e-10)


@pytest.mark.parametrize("m", [40, 150])
def test_rayleigh_ritz_degenerate_spectrum(api, ctx, m):
    """H with a large cluster of zero eigenvalues and repeated nonzero ones (S
    well conditioned): the tridiagonal QL eigensolver must deflate the zero
    cluster (a purely relative test stalls there).  Eigenvalues against
    numpy.linalg.eigh; eigenvectors are not unique inside the clusters, so the
    check is the generalized residual and S-orthonormality."""
    rng = np.random.default_rng(40 + m)
    Q, _ = np.linalg.qr(rng.normal(size=(m, m)))
    w = np.zeros(m)
    w[: m // 4] = np.repeat([3.0, -2.0], (m // 4 + 1) // 2)[: m // 4]
    Hs = (Q * w) @ Q.T
    B = rng.normal(size=(m, m))
    S = B @ B.T / m + np.eye(m)
    L = np.linalg.cholesky(S)
    H = L @ Hs @ L.T  # generalized eigenvalues of (H, S) = w
    nev = m // 2
    ev, V, rank = api.rayleigh_ritz(ctx, to_dev(H[None]), to_dev(S[None]), [m], nev)
    ctx.sync()
    ev, V = ev.cpu().numpy()[0], V.cpu().numpy()[0][:m, :nev]
    ref = np.sort(w)[:nev]
    np.testing.assert_allclose(ev, ref, rtol=0, atol=1e-10)
    res = H @ V - S @ V * ev[None, :]
    assert np.abs(res).max() < 1e-9
    np.testing.assert_allclose(V.T @ S @ V, np.eye(nev), atol=1e-10)


def test_rayleigh_ritz_svqb_rank_deficient(api, ctx):
    rng = np.random.default_rng(3)
    n, m = 40, 12
    Hbig = rng.normal(size=(n, n))
    Hbig = Hbig + Hbig.T
    X = rng.normal(size=(n, m))
    X[:, 11] = X[:, 2]
    H, S = X.T @ Hbig @ X, X.T @ X
    ev, V, rank = api.rayleigh_ritz(ctx, to_dev(H[None]), to_dev(S[None]), [m], 5)
    ctx.sync()
    lam, _, rk = olin.rayleigh_ritz(H, S, 5)
    assert int(rank.cpu()[0]) == rk == 11
    np.testing.assert_allclose(ev.cpu().numpy()[0], lam, atol=1e-8)


def test_rayleigh_ritz_not_pd_reports_error(api, ctx):
    H = np.eye(4)[None]
    S = np.diag([1.0, 1.0, 0.0, 1.0])[None]
    api.rayleigh_ritz(ctx, to_dev(H), to_dev(S), [4], 2, allow_svqb=False)
    with pytest.raises(api.TTNError):
        ctx.sync()


@pytest.mark.parametrize("D", [7, 40])
@pytest.mark.parametrize("dt", [0, 1])
def test_qr_move_matches_oracle(api, ctx, dt, D):
    """QR gauge moves against the oracle's; D=7 keeps every node's matrix in
    LDS, D=40 also sends the 1600 x 40 backbone matrices through the TSQR
    kernels."""
    m = wl.quartic_force_field(8, 21, 20, 30)
    tree = wl.fork_tree(m.dims, 4, 1)
    bonds = wl.bond_dims(tree, D)
    k = 3 if D < 20 else 2
    blk_np = wl.random_block(tree, bonds, k, 44)
    gt = api.Tree(tree.parent, tree.phys)
    tdt = torch.float64 if dt == 0 else torch.float32
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], dt)
    for u in range(tree.n):
        blk.t[u].copy_(to_dev(np.stack([blk_np[j][u] for j in range(k)]), tdt))
    moves = [(5, 4), (4, 0), (0, 1), (1, 2), (2, 3), (3, 10), (10, 11)]
    for (u, v) in moves:
        api.block_move_centre(ctx, blk, u, v)
        for j in range(k):
            ottn.move_centre(tree, blk_np[j], u, v)
    ctx.sync()
    tol = 1e-11 if dt == 0 else 2e-4
    for u in range(tree.n):
        got = blk.t[u].double().cpu().numpy()
        for j in range(k):
            ref = blk_np[j][u]
            assert np.linalg.norm(got[j] - ref) <= tol * max(1.0, np.linalg.norm(ref)), (u, j)


@pytest.mark.parametrize("shape", ["mps_d1", "mps_full", "binary_d3", "chain_tall"])
@pytest.mark.parametrize("dt", [0, 1])
def test_qr_move_edge_shapes(api, ctx, shape, dt):
    """Gauge moves along a whole Euler tour on edge shapes: bond 1 (one
    column, no reflector update), exact bonds where node matrices are square
    (m = n), a ragged binary tree with bond 3, and a 1200 x 2 node matrix (more
    rows than the unrolled LDS instances cover: the runtime-bounded one),
    against the oracle's QR; the absorption of R into the next node runs in
    place."""
    from oracle import ttn as ottn2
    if shape == "binary_d3":
        tree = wl.binary_tree([2, 3, 2, 5, 3])
        D = 3
    elif shape == "chain_tall":
        tree = wl.Tree("chain3", [-1, 0, 1], [2, 40, 30], [0, 1, 2])
        D = 64
    else:
        tree = wl.mps_tree([2, 5, 3, 7, 2], 2)
        D = 1 if shape == "mps_d1" else 64
    bonds = wl.bond_dims(tree, D)
    k = 3
    blk_np = wl.random_block(tree, bonds, k, 46)
    blk_np = [ottn2.canonicalize(tree, st, tree.root) for st in blk_np]
    gt = api.Tree(tree.parent, tree.phys)
    tdt = torch.float64 if dt == 0 else torch.float32
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], dt)
    for u in range(tree.n):
        blk.t[u].copy_(to_dev(np.stack([blk_np[j][u] for j in range(k)]), tdt))
    tour = ottn2.euler_tour(tree)
    for a, b in zip(tour[:-1], tour[1:]):
        api.block_move_centre(ctx, blk, a, b)
        for j in range(k):
            ottn2.move_centre(tree, blk_np[j], a, b)
    ctx.sync()
    tol = 1e-11 if dt == 0 else 2e-4
    for u in range(tree.n):
        got = blk.t[u].double().cpu().numpy()
        for j in range(k):
            ref = blk_np[j][u]
            assert np.linalg.norm(got[j] - ref) <= tol * max(1.0, np.linalg.norm(ref)), (shape, u, j)


def _chain_moves(api, ctx, phys, D, dt, seed):
    """A three-node chain 0 - 1 - 2 (root 0) with the given physical
    dimensions and bond cap D; the centre moves along the Euler tour
    0 -> 1 -> 2 -> 1 -> 0 on the GPU and in the oracle.  Returns the GPU and
    oracle node tensors of every state and the kernels the library recorded
    for the QR and absorption steps ({'qr:m x n' or 'absorb:m x n': name})."""
    tree = wl.Tree("chain3", [-1, 0, 1], list(phys), [0, 1, 2])
    bonds = wl.bond_dims(tree, D)
    k = 2
    blk_np = wl.random_block(tree, bonds, k, seed)
    gt = api.Tree(tree.parent, tree.phys)
    tdt = torch.float64 if dt == 0 else torch.float32
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], dt)
    for u in range(tree.n):
        blk.t[u].copy_(to_dev(np.stack([blk_np[j][u] for j in range(k)]), tdt))
    api.profile(ctx, True)
    paths = {}
    tour = [0, 1, 2, 1, 0]
    for a, b in zip(tour[:-1], tour[1:]):
        api.block_move_centre(ctx, blk, a, b)
        for j in range(k):
            ottn.move_centre(tree, blk_np[j], a, b)
    ctx.sync()
    for r in api.profile_report(ctx):
        if r[0].startswith("qr:") or r[0].startswith("absorb:"):
            paths[r[0]] = r[2]
    api.profile(ctx, False)
    got = [blk.t[u].double().cpu().numpy() for u in range(tree.n)]
    return tree, got, blk_np, paths


@pytest.mark.parametrize("shape", ["1600x40", "1000x40", "1369x37"])
@pytest.mark.parametrize("dt", [0, 1])
def test_tsqr_moves_match_oracle(api, ctx, shape, dt):
    """Node matrices too tall for one workgroup's LDS go through the TSQR
    kernels (row blocks factored in LDS, their stacked R factors factored
    again, the block Q factors multiplied out): 1600 x 40 (the 12-mode
    workload's backbone nodes, four equal blocks), 1000 x 40 (three blocks,
    the last one shorter) and 1369 x 37 (a bond that is not a multiple of the
    eight output columns a thread of the last stage computes).  Against the
    oracle's QR moves, with diag(R) >= 0 the factorisation is unique."""
    phys = {"1600x40": (40, 40, 40), "1000x40": (40, 25, 40), "1369x37": (37, 37, 37)}[shape]
    tree, got, ref, paths = _chain_moves(api, ctx, phys, 40, dt, 52)
    assert paths.get("qr:" + shape) == "tsqr_kernels", paths
    tol = 1e-11 if dt == 0 else 2e-4
    for u in range(tree.n):
        for j in range(len(ref)):
            r = ref[j][u]
            assert np.linalg.norm(got[u][j] - r) <= tol * max(1.0, np.linalg.norm(r)), (shape, u, j)


@pytest.mark.parametrize("phys,D,mat,kernel", [
    ((24, 24, 24), 24, "576x24", "qr_reg_kernel"),   # the c2 interior shape: 9 rows per lane, 2 columns per wave
    ((40, 10, 40), 40, "400x40", "qr_reg_kernel"),   # 7 rows per lane (the 9-row instance), 3 columns per wave
    ((8, 8, 8), 8, "64x8", "qr_reg_kernel"),         # one row per lane, waves 8.. without a column
    ((48, 6, 48), 48, "288x48", "qr_reg_kernel"),    # 48 columns: every wave holds three
    ((17, 4, 17), 17, "68x17", "qr_reg_kernel"),     # 17 columns: wave 0 alone holds two; a ragged second row pass
    ((60, 3, 60), 60, "180x60", "qr_lds_kernel"),    # bond above 48: the LDS-resident kernel
])
@pytest.mark.parametrize("dt", [0, 1])
def test_qr_kernels_by_shape(api, ctx, phys, D, mat, kernel, dt):
    """Each resident-matrix QR kernel on the shape that selects it (the
    register-resident one for up to 576 rows and 48 columns, the LDS-resident
    one beyond), along a whole Euler tour of a three-node chain, against the
    oracle's QR moves."""
    tree, got, ref, paths = _chain_moves(api, ctx, phys, D, dt, 55)
    assert paths.get("qr:" + mat) == kernel, paths
    tol = 1e-11 if dt == 0 else 2e-4
    for u in range(tree.n):
        for j in range(len(ref)):
            r = ref[j][u]
            assert np.linalg.norm(got[u][j] - r) <= tol * max(1.0, np.linalg.norm(r)), (mat, u, j)


@pytest.mark.parametrize("dt", [0, 1])
def test_tsqr_rank_deficient(api, ctx, dt):
    """One move 1 -> 2 on the 40-40-40 chain whose node 1 matrix toward 2
    (1600 x 40) has half its singular values zero, through the TSQR kernels:
    node 1 stays an isometry on the columns that carry weight and the
    two-site tensor of nodes 1 and 2 is unchanged."""
    tree = wl.Tree("chain3", [-1, 0, 1], [40, 40, 40], [0, 1, 2])
    bonds = wl.bond_dims(tree, 40)
    k = 2
    blk_np = wl.random_block(tree, bonds, k, 53)
    rng = np.random.default_rng(9)
    l1, l2 = ottn.leg_of(tree, 1, 2), ottn.leg_of(tree, 2, 1)
    for j in range(k):
        T = np.moveaxis(blk_np[j][1], l1, -1)
        sh = T.shape
        rows, De = int(np.prod(sh[:-1])), sh[-1]
        U, _ = np.linalg.qr(rng.normal(size=(rows, De)))
        V, _ = np.linalg.qr(rng.normal(size=(De, De)))
        sv = np.linspace(1.0, 0.5, De)
        sv[De // 2:] = 0.0
        blk_np[j][1] = np.moveaxis(((U * sv) @ V.T).reshape(sh), -1, l1)
    gt = api.Tree(tree.parent, tree.phys)
    tdt = torch.float64 if dt == 0 else torch.float32
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], dt)
    for u in range(tree.n):
        blk.t[u].copy_(to_dev(np.stack([blk_np[j][u] for j in range(k)]), tdt))
    before = [np.tensordot(blk.t[1][j].double().cpu().numpy(), blk.t[2][j].double().cpu().numpy(),
                           axes=([l1], [l2])) for j in range(k)]
    api.profile(ctx, True)
    api.block_move_centre(ctx, blk, 1, 2)
    ctx.sync()
    paths = {r[0][3:]: r[2] for r in api.profile_report(ctx) if r[0].startswith("qr:")}
    api.profile(ctx, False)
    assert paths.get(f"{rows}x{De}") == "tsqr_kernels", paths
    g1 = blk.t[1].double().cpu().numpy()
    g2 = blk.t[2].double().cpu().numpy()
    eps = 1e-13 if dt == 0 else 3e-6
    for j in range(k):
        Q = np.moveaxis(g1[j], l1, -1).reshape(-1, De)
        G = Q.T @ Q
        nz = np.abs(np.diag(G)) > 0.5
        assert nz.sum() >= De // 2
        assert np.abs(G[np.ix_(nz, nz)] - np.eye(int(nz.sum()))).max() < 50 * eps, j
        after = np.tensordot(g1[j], g2[j], axes=([l1], [l2]))
        assert np.linalg.norm(after - before[j]) <= 50 * eps * np.linalg.norm(before[j]), j


@pytest.mark.parametrize("dt", [0, 1])
def test_qr_global_kernel_shape(api, ctx, dt):
    """A 200 x 98 node matrix (chain 98-2-100): too large for LDS and with a
    bond too wide for TSQR row blocks of at least 98 rows, so the
    global-memory kernel runs; against the oracle's QR moves."""
    tree, got, ref, paths = _chain_moves(api, ctx, (98, 2, 100), 100, dt, 54)
    assert paths.get("qr:200x98") == "qr_kernel", paths
    tol = 1e-11 if dt == 0 else 2e-4
    for u in range(tree.n):
        for j in range(len(ref)):
            r = ref[j][u]
            assert np.linalg.norm(got[u][j] - r) <= tol * max(1.0, np.linalg.norm(r)), (u, j)


@pytest.mark.parametrize("kind", ["cond1e3", "cond1e10", "rank_deficient"])
@pytest.mark.parametrize("dt", [0, 1])
def test_qr_move_conditioning(api, ctx, dt, kind):
    """Gauge moves on node matrices of controlled conditioning (condition
    number 1e3, 1e10, and half the singular values zero): the moved centre is
    an isometry toward v and the two-site tensor of u and v is unchanged; the
    well-conditioned case also matches the oracle's QR."""
    m = wl.quartic_force_field(8, 21, 20, 30)
    tree = wl.fork_tree(m.dims, 4, 1)
    bonds = wl.bond_dims(tree, 7)
    k = 3
    blk_np = wl.random_block(tree, bonds, k, 45)
    u, v = 10, 3  # a 91 x 7 node matrix
    lu, lv = ottn.leg_of(tree, u, v), ottn.leg_of(tree, v, u)
    rng = np.random.default_rng(7)
    if dt == 1 and kind == "cond1e10":
        pytest.skip("FP32 storage rounds such a matrix to a lower rank")
    for j in range(k):
        T = np.moveaxis(blk_np[j][u], lu, -1)
        sh = T.shape
        rows, De = int(np.prod(sh[:-1])), sh[-1]
        U, _ = np.linalg.qr(rng.normal(size=(rows, De)))
        V, _ = np.linalg.qr(rng.normal(size=(De, De)))
        if kind == "cond1e3":
            sv = np.geomspace(1.0, 1e-3, De)
        elif kind == "cond1e10":
            sv = np.geomspace(1.0, 1e-10, De)
        else:
            sv = np.linspace(1.0, 0.5, De)
            sv[De // 2:] = 0.0
        B = (U * sv) @ V.T
        blk_np[j][u] = np.moveaxis(B.reshape(sh), -1, lu)
    gt = api.Tree(tree.parent, tree.phys)
    tdt = torch.float64 if dt == 0 else torch.float32
    blk = api.Block(ctx, gt, k, [max(1, b) for b in bonds], dt)
    for w in range(tree.n):
        blk.t[w].copy_(to_dev(np.stack([blk_np[j][w] for j in range(k)]), tdt))
    before = [np.tensordot(blk_np[j][u], blk_np[j][v], axes=([lu], [lv])) for j in range(k)]
    api.block_move_centre(ctx, blk, u, v)
    ctx.sync()
    gu = blk.t[u].double().cpu().numpy()
    gv = blk.t[v].double().cpu().numpy()
    eps = 1e-13 if dt == 0 else 3e-6
    for j in range(k):
        Q = np.moveaxis(gu[j], lu, -1).reshape(-1, gu[j].shape[lu])
        if kind != "rank_deficient":
            assert np.abs(Q.T @ Q - np.eye(Q.shape[1])).max() < 50 * eps, (kind, j)
        else:
            # columns past the rank carry no weight; those that do stay orthonormal
            G = Q.T @ Q
            nz = np.abs(np.diag(G)) > 0.5
            assert np.abs(G[np.ix_(nz, nz)] - np.eye(int(nz.sum()))).max() < 50 * eps, (kind, j)
        after = np.tensordot(gu[j], gv[j], axes=([lu], [lv]))
        assert np.linalg.norm(after - before[j]) <= 50 * eps * np.linalg.norm(before[j]), (kind, j)
        if kind == "cond1e3":
            ref = [a.copy() for a in blk_np[j]]
            ottn.move_centre(tree, ref, u, v)
            tol = 1e-9 if dt == 0 else 5e-3
            assert np.linalg.norm(gu[j] - ref[u]) <= tol * np.linalg.norm(ref[u]), (kind, j)
            assert np.linalg.norm(gv[j] - ref[v]) <= tol * np.linalg.norm(ref[v]), (kind, j)


def test_node_norms_and_scale(api, ctx):
    tree = wl.binary_tree([3, 4, 5])
    bonds = wl.bond_dims(tree, 4)
    gt = api.Tree(tree.parent, tree.phys)
    blk = api.Block(ctx, gt, 4, [max(1, b) for b in bonds], api.F64)
    for u in range(tree.n):
        blk.t[u].normal_()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    api.block_node_norms2(ctx, blk, 0, out)
    ref = (blk.t[0].reshape(4, -1) ** 2).sum(1)
    ctx.sync()
    np.testing.assert_allclose(out.cpu().numpy(), ref.cpu().numpy(), rtol=1e-13)
    sc = torch.tensor([1.0, 2.0, 0.5, -1.0], dtype=torch.float64, device="cuda")
    before = blk.t[0].clone()
    api.block_scale_node(ctx, blk, 0, sc)
    ctx.sync()
    np.testing.assert_allclose(blk.t[0].cpu().numpy(), (before * sc.view(4, 1, 1, 1)).cpu().numpy(), rtol=1e-15)
