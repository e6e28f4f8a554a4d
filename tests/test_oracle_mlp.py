"""Pins of the oracle's learned-preconditioner network (oracle.mlp): the
hand-derived backward against central finite differences, SiLU at known
points, closed forms of the forward and of Adam's first steps, the tile
feature invariants, and the optimality of the DIAG/learned combination."""
import math

import numpy as np
import pytest

from oracle import mlp


def _loss(p, X, T):
    Y, _ = mlp.forward(p, X)
    return mlp.mse(Y, T)[0]


def test_param_count_and_layout():
    assert mlp.n_params() == 128 * 256 + 256 + 256 * 256 + 256 + 256 * 64 + 64
    p = np.arange(mlp.n_params(), dtype=float)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert W1.shape == (128, 256) and W1[0, 1] == 1 and W1[1, 0] == 256
    assert b1[0] == 128 * 256 and W2[0, 0] == 128 * 256 + 256
    assert b3[-1] == mlp.n_params() - 1


def test_silu_known_values():
    # silu(z) = z * sigmoid(z): sigmoid(1) = e / (1 + e)
    e = math.e
    assert mlp.silu(np.array(0.0)) == 0.0
    assert abs(mlp.silu(np.array(1.0)) - e / (1 + e)) < 1e-15
    assert abs(mlp.silu(np.array(-1.0)) + 1 / (1 + e)) < 1e-15
    assert abs(mlp.dsilu(np.array(0.0)) - 0.5) < 1e-15
    assert abs(mlp.silu(np.array(40.0)) - 40.0) < 1e-12
    # derivative against a central difference
    z = np.linspace(-6, 6, 25)
    fd = (mlp.silu(z + 1e-6) - mlp.silu(z - 1e-6)) / 2e-6
    assert np.max(np.abs(fd - mlp.dsilu(z))) < 1e-9


def test_forward_closed_forms():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(7, 128))
    p = np.zeros(mlp.n_params())
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    b3[:] = np.arange(64)
    Y, _ = mlp.forward(p, X)
    assert np.array_equal(Y, np.tile(np.arange(64.0), (7, 1)))
    # a single path input 5 -> hidden 3 -> hidden 7 -> output 11
    b3[:] = 0
    W1[5, 3] = 2.0
    W2[3, 7] = -1.5
    W3[7, 11] = 0.5
    b1[3] = 0.25
    Y, _ = mlp.forward(p, X)
    s = lambda z: z / (1 + np.exp(-z))
    ref = 0.5 * s(-1.5 * s(2.0 * X[:, 5] + 0.25))
    assert np.max(np.abs(Y[:, 11] - ref)) < 1e-15
    assert np.count_nonzero(np.delete(Y, 11, axis=1)) == 0


@pytest.mark.parametrize("seed", [1, 2])
def test_backward_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    # larger output layer so that every group has O(1) gradients
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    W3 *= 10.0
    b1 += rng.normal(scale=0.3, size=b1.shape)
    b2 += rng.normal(scale=0.3, size=b2.shape)
    X = rng.normal(size=(5, 128))
    T = rng.normal(size=(5, 64))
    Y, cache = mlp.forward(p, X)
    _, dY = mlp.mse(Y, T)
    g = mlp.backward(p, cache, dY)
    # probe parameters from every group: W1, b1, W2, b2, W3, b3
    bounds = np.cumsum([0] + [s for i, o in mlp.SIZES for s in (i * o, o)])
    h = 1e-6
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        for idx in rng.choice(np.arange(lo, hi), size=min(12, hi - lo), replace=False):
            q = p.copy()
            q[idx] += h
            fp = _loss(q, X, T)
            q[idx] -= 2 * h
            fm = _loss(q, X, T)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(g[idx]) * 1e3), (lo, idx, fd, g[idx])
    # the mean-squared error's gradient itself
    fd = np.zeros(5)
    for r in range(5):
        Yp = Y.copy()
        Yp[r, 0] += h
        Ym = Y.copy()
        Ym[r, 0] -= h
        fd[r] = (mlp.mse(Yp, T)[0] - mlp.mse(Ym, T)[0]) / (2 * h)
    assert np.max(np.abs(fd - dY[:, 0])) < 1e-9


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-3
    # bias correction makes the first steps move by lr * g / (|g| + eps) per coordinate
    p1, m, v = mlp.adam_step(p, m, v, g, lr, 1)
    assert np.max(np.abs(p1 - (p - lr * g / (np.abs(g) + 1e-8)))) < 1e-15
    p2, m, v = mlp.adam_step(p1, m, v, g, lr, 2)
    assert np.max(np.abs(p2 - (p1 - lr * g / (np.abs(g) + 1e-8)))) < 1e-14
    # a zero gradient after a step keeps moving along the first moment
    p3, m3, v3 = mlp.adam_step(p2, m, v, np.zeros(50), lr, 3)
    assert np.all(np.sign(p2 - p3) == np.sign(g))


@pytest.mark.parametrize("n", [1, 64, 130, 1000])
def test_features_invariants(n):
    rng = np.random.default_rng(n)
    b = rng.normal(size=n)
    d = rng.uniform(0.5, 3.0, size=n) * rng.choice([-1, 1], size=n)
    X, (nb, sg) = mlp.features(b, d)
    nt = -(-n // 64)
    assert X.shape == (nt, 128)
    bf = X[:, :64].reshape(-1)
    df = X[:, 64:].reshape(-1)
    assert abs(np.sum(bf ** 2) - 1.0) < 1e-13
    assert abs(np.mean(np.abs(df[:n])) - 1.0) < 1e-13
    assert np.count_nonzero(bf[n:]) == 0 and np.count_nonzero(df[n:]) == 0
    assert abs(nb - np.linalg.norm(b)) < 1e-12
    y = rng.normal(size=n)
    Tt = mlp.targets(y, b, d, (nb, sg))
    assert Tt.shape == (nt, 64)
    # the target is the correction over the DIAG step: DIAG + untiled target = y
    assert np.max(np.abs(b / d + mlp.untile(Tt, n, (nb, sg)) - y)) < 1e-12
    assert np.count_nonzero(mlp.targets(b / d, b, d, (nb, sg))) == 0


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return Q @ np.diag(rng.uniform(1.0, 10.0, size=n)) @ Q.T + np.diag(rng.uniform(5, 20, size=n))


def test_mr2_exact_candidate_and_parallel_fallback():
    n = 90
    A = _spd(n, 4)
    rng = np.random.default_rng(5)
    b = rng.normal(size=n)
    yD = b / np.diag(A)
    yL = np.linalg.solve(A, b)
    a, c = mlp.mr2(A @ yD, A @ yL, b)
    assert abs(a) < 1e-10 and abs(c - 1.0) < 1e-10
    # parallel images: c = 0 and the DIAG step's own best scale
    a, c = mlp.mr2(A @ yD, 3.0 * (A @ yD), b)
    Pd = A @ yD
    assert c == 0.0 and abs(a - Pd @ b / (Pd @ Pd)) < 1e-14


def test_mr2_is_optimal_against_brute_force():
    n = 60
    A = _spd(n, 6)
    rng = np.random.default_rng(7)
    b = rng.normal(size=n)
    yD = b / np.diag(A)
    yL = rng.normal(size=n)
    a, c = mlp.mr2(A @ yD, A @ yL, b)
    best = np.linalg.norm(A @ (a * yD + c * yL) - b)
    for aa in np.linspace(a - 0.5, a + 0.5, 41):
        for cc in np.linspace(c - 0.5, c + 0.5, 41):
            assert np.linalg.norm(A @ (aa * yD + cc * yL) - b) >= best - 1e-12
    # never worse than DIAG alone at its best scale
    Pd = A @ yD
    assert best <= np.linalg.norm((Pd @ b / (Pd @ Pd)) * Pd - b) + 1e-12


def test_learned_local_with_zero_network_is_scaled_diag():
    # a network with all-zero parameters outputs zero: y = a * y_D
    n = 70
    A = _spd(n, 8)
    b = np.random.default_rng(9).normal(size=n)
    y, (a, c) = mlp.learned_local(np.zeros(mlp.n_params()), lambda v: A @ v, b, np.diag(A))
    yD = b / np.diag(A)
    Pd = A @ yD
    assert c == 0.0
    assert np.max(np.abs(y - (Pd @ b / (Pd @ Pd)) * yD)) < 1e-14
