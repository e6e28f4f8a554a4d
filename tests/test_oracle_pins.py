"""Pins of the FP64 oracle against facts that do not come from the oracle itself:
textbook closed forms, values printed in the paper, dense / brute-force
references on tiny inputs, library routines for textbook problems, and
invariants.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.linalg

import workloads as wl
from oracle import exact, linalg, operators, solvers, ttn, ttno

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


# ------------------------------------------------------------------ operators

@pytest.mark.parametrize("d", [1, 2, 5, 9, 14])
def test_fbr_harmonic_is_exactly_diagonal(d):
    # textbook: omega/2 (p^2 + q^2) = omega (n + 1/2) in the HO eigenbasis
    q2 = operators.ho_qpow(d, 2)
    p2 = operators.ho_p2(d)
    np.testing.assert_allclose(0.5 * (p2 + q2), np.diag(np.arange(d) + 0.5), atol=1e-13)


def test_q_moments_and_projection():
    # Gaussian ground-state moments <q^2> = 1/2, <q^4> = 3/4, <q^6> = 15/8
    for n, ref in ((2, 0.5), (4, 0.75), (6, 15.0 / 8.0)):
        assert abs(operators.ho_qpow(7, n)[0, 0] - ref) < 1e-13
    # exact projection: the d x d block of q^n does not change with a bigger host basis
    big = np.linalg.matrix_power(operators.ho_q(60), 3)[:8, :8]
    np.testing.assert_allclose(operators.ho_qpow(8, 3), big, atol=1e-12)
    # odd powers are off-diagonal-parity, all are symmetric
    q3 = operators.ho_qpow(6, 3)
    assert np.allclose(q3, q3.T) and np.allclose(np.diag(q3), 0)


def test_dvr_hand_values():
    for N, key in ((1, "dvr_kinetic_N1"), (2, "dvr_kinetic_N2")):
        np.testing.assert_allclose(operators.dvr_kinetic(N), np.array(GOLD[key]["value"]), atol=1e-14)


@pytest.mark.parametrize("N", [3, 6, 8, 9, 14])
def test_dvr_spectrum_law(N):
    # omega/2 (T + X^2) has omega (n + 1/2), n < N-1, plus one level at omega (3N-2)/4
    x = operators.hermite_nodes(N)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (operators.dvr_kinetic(N) + np.diag(x ** 2))))
    ref = np.sort(np.concatenate([np.arange(N - 1) + 0.5, [(3 * N - 2) / 4.0]]))
    np.testing.assert_allclose(ev, ref, atol=1e-11)


# ------------------------------------------------------------------ TTNO

def _tiny_model():
    m = wl.coupled_oscillators(4, 5, 500, 3000, 3, n_cubic=2, name="tiny")
    m.monomials.append(((1, 4),))
    m.coefs = np.append(m.coefs, 2.5)
    m.monomials.append(((0, 1), (2, 2), (3, 1)))
    m.coefs = np.append(m.coefs, -1.25)
    return m


def _tiny_trees(dims):
    return [wl.mps_tree(dims, 1), wl.mps_tree(dims, 0), wl.binary_tree(dims), wl.fork_tree(dims, 2, 1)]


@pytest.mark.parametrize("ti", range(4))
@pytest.mark.parametrize("compress", [False, True])
def test_ttno_equals_kronecker_sop(ti, compress):
    m = _tiny_model()
    tree = _tiny_trees(m.dims)[ti]
    W = ttno.build_ttno(tree, m, compress=compress)
    H = ttno.ttno_to_dense(tree, W)
    Hs = exact.sop_dense_matrix(m)
    assert np.abs(H - Hs).max() <= 1e-12 * np.abs(Hs).max()


def _schmidt_rank(H, dims, inside):
    L = len(dims)
    T = H.reshape(list(dims) + list(dims))
    outside = [i for i in range(L) if i not in inside]
    axes = [i for i in inside] + [L + i for i in inside] + [i for i in outside] + [L + i for i in outside]
    M = np.transpose(T, axes).reshape(int(np.prod([dims[i] ** 2 for i in inside])), -1)
    s = np.linalg.svd(M, compute_uv=False)
    return int(np.sum(s > 1e-12 * s[0]))


@pytest.mark.parametrize("ti", range(4))
def test_ttno_bonds_are_operator_schmidt_ranks(ti):
    m = _tiny_model()
    tree = _tiny_trees(m.dims)[ti]
    W = ttno.build_ttno(tree, m)
    Hs = exact.sop_dense_matrix(m)
    bonds = ttno.ttno_bonds(tree, W)
    for u in range(tree.n):
        if tree.parent[u] < 0:
            continue
        inside = sorted(tree.mode[x] for x in tree.subtree(u) if tree.mode[x] >= 0)
        assert bonds[u] == _schmidt_rank(Hs, m.dims, inside)


def test_paper_64d_model_bond_and_terms():
    m = wl.paper_64d_model()
    assert m.n_terms == GOLD["coupled64_terms"]["value"]
    for tree in (wl.mps_tree(m.dims, 31), wl.binary_tree(m.dims)):
        W = ttno.build_ttno(tree, m)
        assert max(ttno.ttno_bonds(tree, W)) == GOLD["coupled64_max_ttno_bond"]["value"]


def test_c3_term_split_matches_paper_shape():
    m = wl.make_config_model("c3")
    n3 = sum(1 for mono in m.monomials if sum(p for _, p in mono) == 3)
    n4 = sum(1 for mono in m.monomials if sum(p for _, p in mono) == 4)
    assert [m.n_modes, n3, n4] == GOLD["ch3cn_terms"]["value"]


def _product_state(tree, bonds, vecs):
    st = []
    for u in range(tree.n):
        shp = wl.node_shape(tree, bonds, u)
        t = np.zeros(shp)
        idx = tuple([0] * (len(shp) - 1))
        if tree.mode[u] >= 0:
            t[idx] = vecs[tree.mode[u]]
        else:
            t[idx + (0,)] = 1.0
        st.append(t)
    return st


@pytest.mark.parametrize("cfg", ["c2", "c3"])
def test_ttno_product_state_expectation_full_scale(cfg):
    m = wl.make_config_model(cfg)
    tree = wl.binary_tree(m.dims) if cfg == "c2" else wl.fork_tree(m.dims, 4, 1)
    W = ttno.build_ttno(tree, m)
    rng = np.random.default_rng(11)
    vecs = [rng.normal(size=d) for d in m.dims]
    vecs = [v / np.linalg.norm(v) for v in vecs]
    st = _product_state(tree, [1] * tree.n, vecs)
    got = ttn.expectation(tree, st, W, st)
    ref = 0.0
    for i in range(m.n_modes):
        on, _ = operators.mode_operators(m.dims[i], float(m.omega[i]))
        ref += vecs[i] @ on @ vecs[i]
    for mono, c in zip(m.monomials, m.coefs):
        t = c
        for i, p in mono:
            t *= vecs[i] @ operators.ho_qpow(m.dims[i], p) @ vecs[i]
        ref += t
    assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref))


# ------------------------------------------------------------------ environments, H_eff

def _c3_small():
    m = wl.quartic_force_field(8, 21, 20, 30, name="small-qff")
    tree = wl.fork_tree(m.dims, 4, 1)
    return m, tree


def test_closure_independent_of_node_and_edge():
    m, tree = _c3_small()
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 6)
    blk = wl.random_block(tree, bonds, 2, 5)
    vals = [ttn.expectation(tree, blk[0], W, blk[1], at=u) for u in range(tree.n)]
    assert np.ptp(vals) <= 1e-12 * abs(vals[0])
    # on every edge: sum E_{u->v} E_{v->u}
    for u in range(tree.n):
        v = tree.parent[u]
        if v < 0:
            continue
        Eu = ttn.all_envs_toward(tree, v, blk[0], W, blk[1])[(u, v)]
        Ev = ttn.all_envs_toward(tree, u, blk[0], W, blk[1])[(v, u)]
        assert abs(np.sum(Eu * Ev) - vals[0]) <= 1e-12 * abs(vals[0])


def test_identity_environment_of_canonical_state():
    m, tree = _c3_small()
    bonds = wl.bond_dims(tree, 6)
    st = ttn.canonicalize(tree, wl.random_block(tree, bonds, 1, 3)[0], tree.root)
    envs = ttn.all_envs_toward(tree, tree.root, st, None, st)
    for (u, v), E in envs.items():
        np.testing.assert_allclose(E[:, 0, :], np.eye(E.shape[0]), atol=1e-13)


@pytest.mark.parametrize("ti", range(4))
def test_expectation_matches_dense(ti):
    m = _tiny_model()
    tree = _tiny_trees(m.dims)[ti]
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 4)
    blk = wl.random_block(tree, bonds, 2, 9)
    Hs = exact.sop_dense_matrix(m)
    v0, v1 = ttn.to_dense(tree, blk[0]), ttn.to_dense(tree, blk[1])
    assert abs(ttn.expectation(tree, blk[0], W, blk[1]) - v0 @ Hs @ v1) <= 1e-11 * np.abs(Hs).max() * np.linalg.norm(v0) * np.linalg.norm(v1)
    assert abs(ttn.expectation(tree, blk[0], None, blk[1]) - v0 @ v1) <= 1e-12 * np.linalg.norm(v0) * np.linalg.norm(v1)


def test_heff_is_projected_hamiltonian_c1():
    m = wl.make_config_model("c1")
    tree = wl.mps_tree(m.dims, 2)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 8)
    u = 3
    st = ttn.canonicalize(tree, wl.random_block(tree, bonds, 1, 4)[0], u)
    envs = ttn.all_envs_toward(tree, u, st, W, st)
    ein = {c: envs[(c, u)] for c in ttn.nbrs(tree, u)}
    Heff = ttn.heff_dense(tree, u, W[u], ein)
    P = ttn.isometry_at(tree, st, u)
    np.testing.assert_allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-12)
    HP = np.stack([exact.sop_apply_dense(m, P[:, i]) for i in range(P.shape[1])], axis=1)
    ref = P.T @ HP
    assert np.abs(Heff - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.abs(Heff - Heff.T).max() <= 1e-12 * np.abs(Heff).max()
    diag = ttn.heff_diag(tree, u, W[u], ein).ravel()
    np.testing.assert_allclose(diag, np.diag(Heff), atol=1e-10 * np.abs(Heff).max())


# ------------------------------------------------------------------ dense solvers

def test_rayleigh_ritz_matches_generalized_eigh():
    rng = np.random.default_rng(2)
    m = 24
    A = rng.normal(size=(m, m))
    H = A + A.T
    B = rng.normal(size=(m, m))
    S = B @ B.T + m * np.eye(m)
    lam, V, rank = linalg.rayleigh_ritz(H, S, 8)
    ref = scipy.linalg.eigh(H, S, eigvals_only=True)[:8]
    np.testing.assert_allclose(lam, ref, atol=1e-11)
    np.testing.assert_allclose(V.T @ S @ V, np.eye(8), atol=1e-11)
    np.testing.assert_allclose(V.T @ H @ V, np.diag(lam), atol=1e-10)
    assert rank == m
    for j in range(8):
        assert V[np.argmax(np.abs(V[:, j])), j] > 0


def test_rayleigh_ritz_svqb_on_rank_deficient_overlap():
    rng = np.random.default_rng(3)
    n, m = 40, 10
    Hbig = rng.normal(size=(n, n))
    Hbig = Hbig + Hbig.T
    X = rng.normal(size=(n, m))
    X[:, 9] = X[:, 2]  # duplicated direction -> singular S
    H, S = X.T @ Hbig @ X, X.T @ X
    lam, V, rank = linalg.rayleigh_ritz(H, S, 5)
    assert rank == 9
    Q, _ = np.linalg.qr(X[:, :9])
    ref = np.linalg.eigvalsh(Q.T @ Hbig @ Q)[:5]
    np.testing.assert_allclose(lam, ref, atol=1e-9)


def _krylov_minimizer(A, b, k):
    K = np.zeros((len(b), k))
    v = b.copy()
    for i in range(k):
        K[:, i] = v
        v = A @ v
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    return Q @ y


def test_minres_iterates_are_krylov_minimizers():
    rng = np.random.default_rng(4)
    n = 120
    Z = rng.normal(size=(n, n))
    A = Z + Z.T + 0.5 * np.diag(rng.normal(size=n))  # symmetric indefinite
    b = rng.normal(size=n)
    for k in (1, 2, 5, 12):
        x, it, res = linalg.minres(lambda v: A @ v, b, np.zeros(n), 0.0, k)
        xref = _krylov_minimizer(A, b, k)
        assert it == k
        assert np.linalg.norm(x - xref) <= 1e-8 * np.linalg.norm(xref)
        assert abs(res - np.linalg.norm(b - A @ x)) <= 1e-8 * np.linalg.norm(b)


def test_minres_solves_indefinite_system():
    rng = np.random.default_rng(5)
    n = 200
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.concatenate([rng.uniform(-3, -0.5, 80), rng.uniform(0.5, 4, 120)])
    A = Q @ np.diag(ev) @ Q.T
    b = rng.normal(size=n)
    x, it, res = linalg.minres(lambda v: A @ v, b, np.zeros(n), 1e-12, 2000)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-8, atol=1e-9)
    # warm start from the solution: no iteration needed
    x2, it2, _ = linalg.minres(lambda v: A @ v, b, x, 1e-6, 10)
    assert it2 == 0


def test_lanczos_c1_matches_normal_modes():
    m = wl.make_config_model("c1")
    n = int(np.prod(m.dims))
    ev = linalg.lanczos_lowest(lambda v: exact.sop_apply_dense(m, v), n, 10, maxdim=600, tol=1e-12)
    ex = exact.normal_mode_levels(m, 10)
    assert np.max(np.abs(ev - ex)) < 1e-6


def test_normal_modes_match_dense_diagonalisation():
    # 3 modes, large FBR basis: the truncated spectrum converges to the closed form
    m = wl.coupled_oscillators(3, 7, 500, 3000, 18, coupling_scale=0.1)
    H = exact.sop_dense_matrix(m)
    ev = np.linalg.eigvalsh(H)[:10]
    np.testing.assert_allclose(ev, exact.normal_mode_levels(m, 10), atol=1e-6)


# ------------------------------------------------------------------ ALS / fitting

def test_fit_state_to_itself():
    m, tree = _c3_small()
    bonds = wl.bond_dims(tree, 6)
    st = solvers.normalized(tree, wl.random_block(tree, bonds, 1, 8)[0])
    init = solvers.normalized(tree, wl.random_block(tree, bonds, 1, 9)[0])
    y = solvers.fit(tree, [(1.0, None, st)], init, sweeps=2)
    ov = ttn.expectation(tree, y, None, st)
    assert abs(ov - 1.0) < 1e-10
    assert abs(ttn.expectation(tree, y, None, y) - 1.0) < 1e-10


def test_fit_linear_combination_full_bond_is_exact():
    m = _tiny_model()
    tree = wl.binary_tree(m.dims)
    bonds = wl.bond_dims(tree, 100)  # full bonds: the fit is exact
    blk = wl.random_block(tree, bonds, 3, 12)
    W = ttno.build_ttno(tree, m)
    src = [(0.7, W, blk[0]), (-1.3, None, blk[1]), (0.25, None, blk[2])]
    y = solvers.fit(tree, src, blk[2], sweeps=2)
    Hs = exact.sop_dense_matrix(m)
    ref = 0.7 * Hs @ ttn.to_dense(tree, blk[0]) - 1.3 * ttn.to_dense(tree, blk[1]) + 0.25 * ttn.to_dense(tree, blk[2])
    got = ttn.to_dense(tree, y)
    assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


def test_als_full_bond_matches_dense_solve():
    m = _tiny_model()
    tree = wl.mps_tree(m.dims, 1)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 100)
    phi = wl.random_block(tree, bonds, 1, 14)[0]
    Hs = exact.sop_dense_matrix(m)
    s = float(np.linalg.eigvalsh(Hs)[0]) - 300.0  # positive-definite shift
    y = solvers.als_solve(tree, W, s, phi, phi, sweeps=6, maxiter=500, rtol=1e-13)
    ref = np.linalg.solve(Hs - s * np.eye(len(Hs)), ttn.to_dense(tree, phi))
    assert np.linalg.norm(ttn.to_dense(tree, y) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_start_correction_diag_is_exact_for_diagonal_systems():
    """For a diagonal A the DIAG correction reaches the solution in one step
    (r0 / d is the exact correction and its minimal-residual scale is 1)."""
    rng = np.random.default_rng(21)
    d = rng.uniform(0.5, 5.0, size=(4, 5, 3))
    b = rng.normal(size=d.shape)
    y0 = rng.normal(size=d.shape)
    c = solvers.start_correction(lambda v: d * v, b - d * y0, d)
    np.testing.assert_allclose(y0 + c, b / d, rtol=1e-13, atol=1e-13)
    assert not np.any(solvers.start_correction(lambda v: d * v, np.zeros_like(b), d))


def test_start_correction_minimal_residual_scale():
    """On a dense symmetric positive-definite system the DIAG correction's
    residual is no larger than that of the same direction at any other scale
    (brute force over a fine grid), and below |r0|; the learned correction is
    never worse than that scaled DIAG step."""
    from oracle import mlp
    rng = np.random.default_rng(22)
    n = 60
    Z = rng.normal(size=(n, n))
    A = Z @ Z.T / n + np.diag(rng.uniform(1.0, 20.0, n))
    d = np.diag(A).copy()
    r0 = rng.normal(size=n)
    c = solvers.start_correction(lambda v: A @ v, r0, d)
    best = np.linalg.norm(r0 - A @ c)
    g = r0 / d
    grid = [np.linalg.norm(r0 - t * (A @ g)) for t in np.linspace(-1.0, 3.0, 4001)]
    assert best <= min(grid) + 1e-12 and best < np.linalg.norm(r0)
    p = mlp.init_params(3)
    cl = solvers.start_correction(lambda v: A @ v, r0, d, p)
    assert np.linalg.norm(r0 - A @ cl) <= best * (1 + 1e-12)


def test_als_corrected_start_converges_to_dense_solve():
    """Converged ALS from the corrected MINRES starts reaches the same exact
    solution as the plain method."""
    m = _tiny_model()
    tree = wl.mps_tree(m.dims, 1)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 100)
    phi = wl.random_block(tree, bonds, 1, 14)[0]
    Hs = exact.sop_dense_matrix(m)
    s = float(np.linalg.eigvalsh(Hs)[0]) - 300.0
    ref = np.linalg.solve(Hs - s * np.eye(len(Hs)), ttn.to_dense(tree, phi))
    y = solvers.als_solve(tree, W, s, phi, phi, sweeps=6, maxiter=500, rtol=1e-13, local="minres+diag")
    assert np.linalg.norm(ttn.to_dense(tree, y) - ref) <= 1e-8 * np.linalg.norm(ref)


# ------------------------------------------------------------------ eigensolvers

def test_clusters_single_linkage():
    lam = np.array([10.0, 3.0, 4.0, 30.0, 8.9, 33.5])
    cl = solvers.clusters_of(lam, 5.0)
    assert [sorted(c) for c in cl] == [[1, 2, 4, 0], [3, 5]] or [sorted(c) for c in cl] == [[0, 1, 2, 4], [3, 5]]


def test_uncoupled_product_states_are_exact_at_bond_one():
    # c = 0: the lowest product states are exact eigenstates; their energies
    # sum_i omega_i n_i (shifted frame) come out of the TTNO expectation
    m = wl.make_config_model("c1")
    m.monomials, m.coefs = [], np.zeros(0)
    tree = wl.mps_tree(m.dims, 2)
    W = ttno.build_ttno(tree, m)
    occ = wl.lowest_product_states(m.omega, m.dims, 6)
    for n in occ:
        vecs = [np.eye(d)[n[i]] for i, d in enumerate(m.dims)]
        st = _product_state(tree, [1] * tree.n, vecs)
        assert abs(ttn.expectation(tree, st, W, st) - float(np.dot(m.omega, n))) < 1e-10


@pytest.mark.slow
def test_lobpcg_c1_reaches_closed_form():
    m = wl.make_config_model("c1")
    tree = wl.mps_tree(m.dims, 2)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 8)
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, 10, m.seed + 17)
    lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
    opts = solvers.LobpcgOptions(n_iter=7, shift=float(np.min(lam0)) - 837.0)
    xs, lam = solvers.lobpcg(tree, W, x0, opts)
    ex = exact.normal_mode_levels(m, 10)
    lam = np.sort(lam)
    assert np.max(np.abs(lam - ex)) < 1e-3
    assert np.all(lam >= ex - 1e-9)  # variational (Galerkin) bound


def _near_degenerate_model():
    """Three modes whose two fundamentals lie 2.5 cm^-1 apart and are mixed by
    a bilinear coupling (2 x 2 block [[1000, 1], [1, 1002.5]] in the
    {|100>, |010>} pair: levels 2.5 +- 3.2 cm^-1 apart after mixing), plus
    couplings to the third mode and a cubic term."""
    omega = np.array([1000.0, 1002.5, 1500.0])
    monos = [((0, 1), (1, 1)), ((1, 1), (2, 1)), ((0, 1), (2, 1)), ((0, 2), (2, 1))]
    coefs = np.array([2.0, 15.0, -9.0, 4.0])
    return wl.SOPModel("near_degenerate", omega, [4, 4, 4], monos, coefs, 0)


def _dense_block_inverse_iteration(H, X, lam, clusters):
    """One outer iteration of Alg. block_inverse_iteration on dense vectors:
    per cluster, s = mean Rayleigh quotient, x_j <- (H - s)^{-1} x_j
    normalised, then (clusters of more than one state) the cluster's
    generalized eigenproblem and x_j <- sum_k V[k, j] x_k, normalised."""
    X = [x.copy() for x in X]
    n = len(H)
    for c in clusters:
        s = sum(float(lam[j]) for j in c) / len(c)
        for j in c:
            y = np.linalg.solve(H - s * np.eye(n), X[j])
            X[j] = y / np.linalg.norm(y)
        if len(c) > 1:
            B = np.stack([X[j] for j in c], axis=1)
            _, V = scipy.linalg.eigh(B.T @ H @ B, B.T @ B)
            newx = [B @ V[:, jj] for jj in range(len(c))]
            for jj, j in enumerate(c):
                X[j] = newx[jj] / np.linalg.norm(newx[jj])
    return X, np.array([x @ H @ x for x in X])


def test_inverse_iteration_full_bond_near_degenerate_pair():
    """Full bond dimension, so one ALS sweep solves the shifted system exactly
    and the fits are exact: every outer iteration of the oracle must equal the
    same iteration done on dense vectors (brute force, 64 dimensions),
    including the in-cluster Rayleigh-Ritz of the near-degenerate pair, and
    the final Ritz values must reach the dense eigenvalues.  Two outer
    iterations: a third would shift a converged singleton by its own
    eigenvalue to ~1e-10, where (H - s) is numerically singular and MINRES
    cannot meet its tolerance (a degenerate case of the algorithm itself)."""
    m = _near_degenerate_model()
    tree = wl.mps_tree(m.dims, 1)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 100)
    k = 4
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, k, 33)
    xs = [solvers.normalized(tree, x) for x in x0]
    lam0 = solvers.rayleigh_quotients(tree, W, xs)
    cl = solvers.clusters_of(lam0, 5.0)
    assert sorted(len(c) for c in cl) == [1, 1, 2]  # the pair shares one shift
    assert solvers.IIOptions().monotone is False     # Alg. block_inverse_iteration as printed by default
    hist = []
    _, theta = solvers.inverse_iteration(tree, W, xs, lam0, solvers.IIOptions(n_iter=2), hist)
    H = exact.sop_dense_matrix(m)
    X = [ttn.to_dense(tree, x) for x in xs]
    lam = lam0.copy()
    for it in range(2):
        X, lam = _dense_block_inverse_iteration(H, X, lam, cl)
        np.testing.assert_allclose(hist[it]["lam"], lam, rtol=0, atol=1e-7)
    ev = np.linalg.eigvalsh(H)[:k]
    np.testing.assert_allclose(theta, ev, rtol=0, atol=1e-8)
    assert np.all(theta >= ev - 1e-9)


@pytest.mark.slow
def test_lobpcg_then_inverse_iteration_c1_reaches_closed_form():
    """c1: three LOBPCG iterations, then two outer iterations of block inverse
    iteration and the final global Rayleigh-Ritz: every level within 1e-3
    cm^-1 of the normal-mode closed form and variationally above it."""
    m = wl.make_config_model("c1")
    tree = wl.mps_tree(m.dims, 2)
    W = ttno.build_ttno(tree, m)
    bonds = wl.bond_dims(tree, 8)
    x0 = wl.initial_block(tree, bonds, m.omega, m.dims, 10, m.seed + 17)
    lam0 = solvers.rayleigh_quotients(tree, W, [solvers.normalized(tree, x) for x in x0])
    xs, lam = solvers.lobpcg(tree, W, x0, solvers.LobpcgOptions(n_iter=3, shift=float(np.min(lam0)) - 837.0))
    _, theta = solvers.inverse_iteration(tree, W, xs, lam, solvers.IIOptions(n_iter=2))
    ex = exact.normal_mode_levels(m, 10)
    assert np.max(np.abs(theta - ex)) < 1e-3
    assert np.all(theta >= ex - 1e-7)


# ------------------------------------------------------------------ SRC

@pytest.mark.parametrize("kind", ["mps", "binary", "fork"])
def test_src_recovers_product_exactly_at_full_sketch(kind):
    """Successive randomized compression (Sec. II.C.1): once the sketch size
    chi reaches the rank of every unfolding of H x, the randomized range
    finder captures the range exactly (Gaussian test matrices), so the
    compressed state equals the dense product H x; every non-root tensor is
    an isometry toward its parent (canonical at the root); below that rank
    the error is nonzero and the bonds never exceed chi."""
    from oracle import src
    m = wl.coupled_oscillators(4, 5, 500, 3000, 3, n_cubic=2)
    tree = {"mps": wl.mps_tree(m.dims, 1), "binary": wl.binary_tree(m.dims), "fork": wl.fork_tree(m.dims, 2, 1)}[kind]
    W = ttno.build_ttno(tree, m)
    x = wl.random_block(tree, [max(1, b) for b in wl.bond_dims(tree, 2)], 1, 3)[0]
    ref = exact.sop_dense_matrix(m) @ ttn.to_dense(tree, x)
    rng = np.random.default_rng(1)
    for chi, tol in ((3, None), (9, 1e-12), (20, 1e-12)):
        om = [rng.normal(size=(tree.phys[u], chi)) for u in range(tree.n)]
        y, bonds = src.src_apply(tree, W, x, om, chi)
        err = np.linalg.norm(ttn.to_dense(tree, y) - ref) / np.linalg.norm(ref)
        assert max(bonds) <= chi
        if tol is None:
            assert err > 1e-6
        else:
            assert err < tol, (chi, err)
        for u in range(tree.n):
            if u != tree.root:
                Q = y[u].reshape(y[u].shape[0], -1)
                np.testing.assert_allclose(Q @ Q.T, np.eye(Q.shape[0]), atol=1e-12)
        assert abs(np.linalg.norm(y[tree.root]) - np.linalg.norm(ttn.to_dense(tree, y))) < 1e-12 * np.linalg.norm(ref)


def test_src_of_identity_operator_returns_the_state():
    """With the identity as operator and chi at least the state's bonds, SRC
    returns the state itself (in its canonical gauge)."""
    from oracle import src
    m = wl.make_config_model("c3")
    tree = wl.fork_tree(m.dims, 4, 1)
    bonds = [max(1, b) for b in wl.bond_dims(tree, 3)]
    x = wl.random_block(tree, bonds, 1, 8)[0]
    Wid = [ttn.identity_op(tree, u) for u in range(tree.n)]
    rng = np.random.default_rng(2)
    om = [rng.normal(size=(tree.phys[u], 3)) for u in range(tree.n)]
    y, yb = src.src_apply(tree, Wid, x, om, 3)
    ov = ttn.expectation(tree, y, None, x)
    nx = ttn.expectation(tree, x, None, x)
    assert abs(ov - nx) < 1e-10 * nx
    assert abs(ttn.expectation(tree, y, None, y) - nx) < 1e-10 * nx


# ------------------------------------------------------------- bond expansion (Sec. II.C.2, III.B)

def _expansion_trees(dims):
    return {"mps": wl.mps_tree(dims, 1), "binary": wl.binary_tree(dims), "fork": wl.fork_tree(dims, 2, 1)}


@pytest.mark.parametrize("kind", ["mps", "binary", "fork"])
def test_expansion_keeps_the_state(kind):
    """Growing every bond (1 -> up to 9) keeps the state exactly, every
    non-root tensor an isometry toward its parent, the bonds as requested."""
    from oracle import expand
    m = wl.coupled_oscillators(4, 5, 500, 3000, 3, n_cubic=2)
    tree = _expansion_trees(m.dims)[kind]
    W = ttno.build_ttno(tree, m)
    lo = [max(1, b) for b in wl.bond_dims(tree, 1)]
    hi = [max(1, b) for b in wl.bond_dims(tree, 9)]
    x = ttn.canonicalize(tree, wl.random_block(tree, lo, 1, 3)[0], tree.root)
    y = expand.expand_bonds(tree, W, x, hi, wl.sketch_matrices(tree, 10, 4), 10)
    dx, dy = ttn.to_dense(tree, x), ttn.to_dense(tree, y)
    assert np.linalg.norm(dy - dx) < 1e-12 * np.linalg.norm(dx)
    for u in range(tree.n):
        if u == tree.root:
            continue
        assert y[u].shape[0] == hi[u]
        Y = y[u].reshape(hi[u], -1)
        assert np.abs(Y @ Y.T - np.eye(hi[u])).max() < 1e-12


def _grown_basis(tree, y):
    """Dense images of the root's unit tensors: the span of states that share
    y's non-root tensors."""
    r = tree.root
    cols = []
    for i in range(y[r].size):
        e = np.zeros(y[r].size)
        e[i] = 1.0
        z = list(y)
        z[r] = e.reshape(y[r].shape)
        cols.append(ttn.to_dense(tree, z))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("kind", ["mps", "binary", "fork"])
def test_expansion_captures_hx_of_a_one_body_model(kind):
    """For a Hamiltonian of one-body terms and a product state x, H x has
    Schmidt rank 2 across every edge (x on one side, the one-body part applied
    on the other), so growing every bond from 1 by one direction must make H x
    exactly representable in the grown basis.  A wrong leg, a stale <y|H|x>
    environment or a missing projection leaves part of H x outside."""
    from oracle import expand
    rng = np.random.default_rng(11)
    L = 4
    model = wl.SOPModel("one-body", omega=np.array([700.0, 1300.0, 1900.0, 2600.0]), dims=[3] * L,
                        monomials=[((i, 1),) for i in range(L)] + [((i, 3),) for i in range(L)],
                        coefs=rng.normal(0.0, 30.0, size=2 * L))
    tree = _expansion_trees(model.dims)[kind]
    W = ttno.build_ttno(tree, model)
    one = [1] * tree.n
    two = [max(1, b) for b in wl.bond_dims(tree, 2)]
    x = ttn.canonicalize(tree, wl.random_block(tree, one, 1, 5)[0], tree.root)
    y = expand.expand_bonds(tree, W, x, two, wl.sketch_matrices(tree, 2, 6), 2)
    h = exact.sop_dense_matrix(model) @ ttn.to_dense(tree, x)
    Phi = _grown_basis(tree, y)
    proj = Phi @ (Phi.T @ h)
    assert np.linalg.norm(proj - h) < 1e-10 * np.linalg.norm(h)
    # without growth H x is not representable (the test is not vacuous)
    Phi0 = _grown_basis(tree, x)
    assert np.linalg.norm(Phi0 @ (Phi0.T @ h) - h) > 1e-3 * np.linalg.norm(h)


def test_pivoted_completion_reduces_to_lapack_pivoted_qr():
    """With the leading block Q and a sketch S of full rank, the completion is
    the column-pivoted QR (LAPACK dgeqp3) of S projected outside span(Q):
    same pivot order, same orthonormal columns once diag(R) >= 0."""
    import scipy.linalg
    from oracle import expand
    rng = np.random.default_rng(3)
    m, D, n, grow = 40, 5, 9, 7
    Q, _ = np.linalg.qr(rng.normal(size=(m, D)))
    S = rng.normal(size=(m, n)) * np.linspace(1.0, 3.0, n)[None, :]
    P = expand.pivoted_completion(Q, S, grow)
    Sp = S - Q @ (Q.T @ S)
    Qs, Rs, _ = scipy.linalg.qr(Sp, mode="economic", pivoting=True)
    ref = Qs[:, :grow] * np.where(np.diag(Rs)[:grow] < 0, -1.0, 1.0)[None, :]
    assert np.abs(P - ref).max() < 1e-12
    assert np.abs(Q.T @ P).max() < 1e-13


# ------------------------------------------------------------- state-diagram TTNO (Sec. II.A.3)

@pytest.mark.parametrize("case", [(4, 3, 2), (5, 2, 4), (6, 2, 10)])
@pytest.mark.parametrize("kind", ["mps", "binary", "fork"])
def test_state_diagram_ttno_is_the_sop_operator(case, kind):
    """The state-diagram TTNO contracts to the Kronecker sum of products on
    tiny trees (chains and branching trees; without the forced
    coefficient-free channels of merged items the branching trees fail by
    ~2e3 relative), and its bonds are the operator Schmidt ranks (SVD of the
    dense operator's bipartitions, via the compressed build) -- terms with
    generic coefficients have no algebraic shortcut that a vertex cover
    misses."""
    from oracle import statediagram as sd
    L, d, nc = case
    m = wl.coupled_oscillators(L, L + 3, 500, 3000, d, n_cubic=nc)
    tree = {"mps": wl.mps_tree(m.dims, 1), "binary": wl.binary_tree(m.dims), "fork": wl.fork_tree(m.dims, 2, 1)}[kind]
    W = sd.state_diagram_ttno(tree, m)
    H = exact.sop_dense_matrix(m)
    assert np.abs(ttno.ttno_to_dense(tree, W) - H).max() < 1e-13 * np.abs(H).max()
    assert ttno.ttno_bonds(tree, W) == ttno.ttno_bonds(tree, ttno.build_ttno(tree, m))


def test_min_vertex_cover_against_brute_force():
    """Konig's cover from the augmenting-path matching is a vertex cover of
    minimum size (all subsets enumerated on random bipartite graphs up to
    6 + 6 vertices), also with forced left vertices."""
    import itertools
    from oracle import statediagram as sd
    rng = np.random.default_rng(5)
    for trial in range(200):
        nl, nr = rng.integers(1, 7, size=2)
        adj = [sorted(set(rng.choice(nr, size=rng.integers(0, nr + 1), replace=True).tolist())) for _ in range(nl)]
        forced = [l for l in range(nl) if rng.random() < 0.2]
        cl, cr = sd.min_vertex_cover(nl, nr, adj, forced)
        edges = [(l, r) for l in range(nl) for r in adj[l]]
        assert all(l in cl or r in cr for l, r in edges), trial
        assert set(forced) <= set(cl)
        best = None
        verts = [("l", l) for l in range(nl) if l not in forced] + [("r", r) for r in range(nr)]
        for size in range(len(verts) + 1):
            for S in itertools.combinations(verts, size):
                L = set(forced) | {v for t, v in S if t == "l"}
                R = {v for t, v in S if t == "r"}
                if all(l in L or r in R for l, r in edges):
                    best = len(L) + len(R)
                    break
            if best is not None:
                break
        assert len(cl) + len(cr) == best, (trial, nl, nr, adj, forced)
