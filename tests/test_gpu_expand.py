"""Bond expansion on the GPU (ttn_expand_*) against the oracle's
expand_bonds with the same Khatri-Rao sketch matrices (drawn by
workloads.sketch_matrices, passed to both sides): node by node in FP64, and
the properties that hold at any precision (the state is kept, every non-root
tensor is an isometry, a one-body H x becomes representable)."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import exact
from oracle import expand as oexp
from oracle import ttn as ottn
from oracle import ttno as ottno
from tests.gpu_util import rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    ttn.lib()
    return ttn


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0, workspace_bytes=1 << 30)


def _gpu_expand(api, ctx, tree, W, M, xs, lo, hi, n, om, dt):
    """xs: k host states with bonds lo; om[u]: [d_u x n] sketch matrices (oracle layout)."""
    tdt = torch.float64 if dt == api.F64 else torch.float32
    gt = api.Tree(tree.parent, tree.phys)
    op = api.TTNO(ctx, gt, [to_dev(w, tdt) for w in W], [max(1, x) for x in M], dt)
    k = len(xs)
    X = api.Block(ctx, gt, k, lo, dt)
    for u in range(tree.n):
        X.t[u].copy_(to_dev(np.stack([xs[j][u] for j in range(k)]), tdt))
    Y = api.Block(ctx, gt, k, hi, dt)
    e = api.Expand(ctx, gt, op, X, Y, n, dt)
    e.apply([to_dev(np.ascontiguousarray(om[u].T), tdt) if om[u] is not None else None for u in range(tree.n)])
    ctx.sync()
    out = [[Y.t[u][j].double().cpu().numpy().reshape(Y.legdims(u)) for u in range(tree.n)] for j in range(k)]
    e.close()
    return out


def _trees(dims):
    return {"mps": wl.mps_tree(dims, 1), "binary": wl.binary_tree(dims), "fork": wl.fork_tree(dims, 2, 1)}


def _isometry_err(tree, y):
    return max(np.abs(y[u].reshape(y[u].shape[0], -1) @ y[u].reshape(y[u].shape[0], -1).T
                      - np.eye(y[u].shape[0])).max() for u in range(tree.n) if u != tree.root)


def _compare_determined(tree, yg, yo, info, tol):
    """Node by node: the kept basis and the determined completions (info from
    the oracle) equal; beyond the sketch's rank the completions are arbitrary
    orthonormal directions on both sides (checked by the isometry test), and
    they carry no weight, so the root is compared whole."""
    for u in range(tree.n):
        if u == tree.root:
            assert rel_err(yg[u], yo[u]) < tol, u
            continue
        D, r = info[u]
        G = yg[u].reshape(yg[u].shape[0], -1)[:D + r]
        O = yo[u].reshape(yo[u].shape[0], -1)[:D + r]
        assert rel_err(G, O) < tol, (u, D, r)


@pytest.mark.parametrize("kind", ["mps", "binary", "fork"])
@pytest.mark.parametrize("bonds", [(1, 9), (2, 5)])
def test_expand_matches_oracle_small_trees(api, ctx, kind, bonds):
    """Bonds grown 1 -> 9 (the residual of a product state has low rank: most
    completions beyond it) and 2 -> 5 on three small trees (4 modes, d = 3),
    two states: the kept bases, the determined completions and the root equal
    the oracle's to 1e-10; y equals x as a vector; every node an isometry."""
    m = wl.coupled_oscillators(4, 5, 500, 3000, 3, n_cubic=2)
    tree = _trees(m.dims)[kind]
    W = ottno.build_ttno(tree, m)
    M = ottno.ttno_bonds(tree, W)
    lo = [max(1, b) for b in wl.bond_dims(tree, bonds[0])]
    hi = [max(1, b) for b in wl.bond_dims(tree, bonds[1])]
    n = 10
    xs = [ottn.canonicalize(tree, x, tree.root) for x in wl.random_block(tree, lo, 2, 3)]
    om = wl.sketch_matrices(tree, n, 4)
    ys = _gpu_expand(api, ctx, tree, W, M, xs, lo, hi, n, om, api.F64)
    for j in range(2):
        info = {}
        yo = oexp.expand_bonds(tree, W, xs[j], hi, om, n, info)
        _compare_determined(tree, ys[j], yo, info, 1e-10)
        assert rel_err(ottn.to_dense(tree, ys[j]), ottn.to_dense(tree, xs[j])) < 1e-12
        assert _isometry_err(tree, ys[j]) < 1e-12


@pytest.mark.parametrize("dt", [0, 1])
def test_expand_fork4_force_field(api, ctx, dt):
    """The 12-mode quartic force field on the fork-4 comb, three states grown
    from D = 4 to D = 7 with 5 sketch columns (every completion determined):
    FP64 node by node against the oracle at 1e-9; FP32 (its pivot choices may differ from FP64 where column
    norms agree to FP32 rounding) through the properties that fix no gauge:
    y = x as states and every non-root tensor an isometry, both to 1e-5."""
    m = wl.make_config_model("c3")
    tree = wl.fork_tree(m.dims, 4, 1)
    W = ottno.build_ttno(tree, m)
    M = ottno.ttno_bonds(tree, W)
    lo = [max(1, b) for b in wl.bond_dims(tree, 4)]
    hi = [max(1, b) for b in wl.bond_dims(tree, 7)]
    xs = [ottn.canonicalize(tree, x, tree.root) for x in wl.random_block(tree, lo, 3, 8)]
    om = wl.sketch_matrices(tree, 5, 9)
    ys = _gpu_expand(api, ctx, tree, W, M, xs, lo, hi, 5, om, dt)
    for j in range(3):
        if dt == 0:
            info = {}
            yo = oexp.expand_bonds(tree, W, xs[j], hi, om, 5, info)
            assert all(r == hi[u] - D for u, (D, r) in info.items()), info  # full-rank residual sketches
            _compare_determined(tree, ys[j], yo, info, 1e-9)
        aa = ottn.expectation(tree, ys[j], None, ys[j])
        bb = ottn.expectation(tree, xs[j], None, xs[j])
        ab = ottn.expectation(tree, ys[j], None, xs[j])
        # |y - x| from overlaps: the difference of FP64 sums of size |x|^2 has a
        # floor near sqrt(1e-16) = 1e-8 relative
        assert np.sqrt(max(aa + bb - 2 * ab, 0.0) / bb) < (1e-7 if dt == 0 else 1e-5), j
        assert _isometry_err(tree, ys[j]) < (1e-12 if dt == 0 else 1e-5), j


@pytest.mark.parametrize("kind", ["mps", "binary"])
def test_expand_captures_hx_of_a_one_body_model(api, ctx, kind):
    """One-body Hamiltonian, product state, every bond grown by one direction:
    H x lies in the span of the grown basis (the GPU counterpart of the oracle
    pin)."""
    rng = np.random.default_rng(11)
    L = 4
    model = wl.SOPModel("one-body", omega=np.array([700.0, 1300.0, 1900.0, 2600.0]), dims=[3] * L,
                        monomials=[((i, 1),) for i in range(L)] + [((i, 3),) for i in range(L)],
                        coefs=rng.normal(0.0, 30.0, size=2 * L))
    tree = _trees(model.dims)[kind]
    W = ottno.build_ttno(tree, model)
    M = ottno.ttno_bonds(tree, W)
    one = [1] * tree.n
    two = [max(1, b) for b in wl.bond_dims(tree, 2)]
    x = ottn.canonicalize(tree, wl.random_block(tree, one, 1, 5)[0], tree.root)
    y = _gpu_expand(api, ctx, tree, W, M, [x], one, two, 2, wl.sketch_matrices(tree, 2, 6), api.F64)[0]
    h = exact.sop_dense_matrix(model) @ ottn.to_dense(tree, x)
    r = tree.root
    cols = []
    for i in range(y[r].size):
        e = np.zeros(y[r].size)
        e[i] = 1.0
        z = list(y)
        z[r] = e.reshape(y[r].shape)
        cols.append(ottn.to_dense(tree, z))
    Phi = np.stack(cols, axis=1)
    assert np.linalg.norm(Phi @ (Phi.T @ h) - h) < 1e-10 * np.linalg.norm(h)
