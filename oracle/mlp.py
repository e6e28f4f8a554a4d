"""The learned local preconditioner (oracle, FP64 NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not part of the paper's method: its outlook names better preconditioners as
future work, and this network is one.  What it computes:

* tiles: a local vector of n entries is cut into T = 64 consecutive entries
  per tile, the last tile zero-padded;
* features of a tile of state j: [b_tile / |b_j|, d_tile / sigma_j], with
  d = diag(H_eff) - s_j and sigma_j = mean |d| over the node (reading: the
  mean rather than a median, one reduction pass);
* network: x -> silu(x W1 + b1) -> silu(. W2 + b2) -> . W3 + b3, widths
  128 -> 256 -> 256 -> 64, silu(z) = z / (1 + exp(-z)); parameters packed
  row-major as W1[128][256], b1, W2[256][256], b2, W3[256][64], b3;
* output: the correction to the DIAG step b / d, in units of |b_j| / sigma_j
  (training targets (y - b/d) sigma_j / |b_j| for a MINRES solution y);
* loss: mean squared error over all outputs; optimiser: Adam with bias
  correction;
* local step (LEARNED): y_D = b / d (the diagonal preconditioner), y_L the
  network's correction; the result is a y_D + c y_L with (a, c) the least
  squares minimiser of |A (a y_D + c y_L) - b| for the shifted local operator
  A = H_eff - s; c = 0 and a = <A y_D, b> / |A y_D|^2 when the two images are
  numerically parallel (Gram determinant <= 1e-10 of the product of the
  squared norms).

The backward pass is derived by hand from the chain rule (no autodiff) and is
pinned against central finite differences of the loss.
"""
from __future__ import annotations

from typing import Callable, Dict, Tuple

import numpy as np

T_TILE = 64
SIZES = [(128, 256), (256, 256), (256, 64)]


def n_params() -> int:
    return sum(i * o + o for i, o in SIZES)


def unpack(p: np.ndarray):
    """Views (W1, b1, W2, b2, W3, b3) into the packed parameter vector."""
    out, off = [], 0
    for i, o in SIZES:
        out.append(p[off:off + i * o].reshape(i, o))
        off += i * o
        out.append(p[off:off + o])
        off += o
    return out


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation with small output layer (a seeded draw)."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (i, o) in enumerate(SIZES):
        scale = np.sqrt(2.0 / i) * (0.1 if li == len(SIZES) - 1 else 1.0)
        parts += [rng.normal(scale=scale, size=i * o), np.zeros(o)]
    return np.concatenate(parts)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s + z * s * (1.0 - s)


def forward(p: np.ndarray, X: np.ndarray) -> Tuple[np.ndarray, Dict[str, np.ndarray]]:
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z1 = X @ W1 + b1
    h1 = silu(z1)
    z2 = h1 @ W2 + b2
    h2 = silu(z2)
    Y = h2 @ W3 + b3
    return Y, {"X": X, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def backward(p: np.ndarray, cache: Dict[str, np.ndarray], dY: np.ndarray) -> np.ndarray:
    """Gradient of sum(dY * Y) with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X, z1, h1, z2, h2 = cache["X"], cache["z1"], cache["h1"], cache["z2"], cache["h2"]
    gW3 = h2.T @ dY
    gb3 = dY.sum(axis=0)
    g2 = (dY @ W3.T) * dsilu(z2)
    gW2 = h1.T @ g2
    gb2 = g2.sum(axis=0)
    g1 = (g2 @ W2.T) * dsilu(z1)
    gW1 = X.T @ g1
    gb1 = g1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def mse(Y: np.ndarray, T: np.ndarray) -> Tuple[float, np.ndarray]:
    """Mean squared error and its gradient with respect to Y."""
    diff = Y - T
    return float(np.mean(diff * diff)), 2.0 * diff / diff.size


def adam_step(p, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (returns new p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(b: np.ndarray, d: np.ndarray):
    """Tile features of one state's local vectors b, d (flat, length n):
    X[ntiles][128] and the scales (|b|, sigma)."""
    n = b.size
    nt = -(-n // T_TILE)
    nb = float(np.linalg.norm(b))
    sg = float(np.mean(np.abs(d))) if n else 0.0
    bp = np.zeros(nt * T_TILE)
    dp = np.zeros(nt * T_TILE)
    bp[:n] = b / nb if nb > 0 else 0.0
    dp[:n] = d / sg if sg > 0 else 0.0
    return np.concatenate([bp.reshape(nt, T_TILE), dp.reshape(nt, T_TILE)], axis=1), (nb, sg)


def targets(y: np.ndarray, b: np.ndarray, d: np.ndarray, scales) -> np.ndarray:
    """Training target of a solution y: its correction over the DIAG step in
    network units, (y - b / d) * sigma / |b| (0 where d = 0)."""
    nb, sg = scales
    n = y.size
    nt = -(-n // T_TILE)
    yp = np.zeros(nt * T_TILE)
    if nb > 0:
        yd = np.divide(b, d, out=np.zeros(n), where=d != 0)
        yp[:n] = (y - yd) * sg / nb
    return yp.reshape(nt, T_TILE)


def untile(Yn: np.ndarray, n: int, scales) -> np.ndarray:
    """Network output tiles back to a local vector: out * |b| / sigma."""
    nb, sg = scales
    if not sg > 0:
        return np.zeros(n)
    return Yn.reshape(-1)[:n] * nb / sg


def learned_candidate(p: np.ndarray, b: np.ndarray, d: np.ndarray) -> np.ndarray:
    X, sc = features(b, d)
    Yn, _ = forward(p, X)
    return untile(Yn, b.size, sc)


def mr2(Pd: np.ndarray, Pl: np.ndarray, b: np.ndarray) -> Tuple[float, float]:
    """(a, c) minimising |a Pd + c Pl - b|; (<Pd, b>/|Pd|^2, 0) when Pd and Pl
    are numerically parallel."""
    dd, dl, ll = Pd @ Pd, Pd @ Pl, Pl @ Pl
    a = float(Pd @ b / dd) if dd > 0 else 1.0
    c = 0.0
    det = dd * ll - dl * dl
    if np.isfinite(det) and det > 1e-10 * dd * ll:
        # least squares on the two columns [Pd, Pl] (library solver)
        coef, *_ = np.linalg.lstsq(np.stack([Pd, Pl], axis=1), b, rcond=None)
        a, c = float(coef[0]), float(coef[1])
    return a, c


def learned_local(p: np.ndarray, apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, d: np.ndarray):
    """LEARNED local step on flat vectors: returns (y, (a, c))."""
    yD = b / d
    yL = learned_candidate(p, b, d)
    a, c = mr2(apply_A(yD), apply_A(yL), b)
    return a * yD + c * yL, (a, c)
