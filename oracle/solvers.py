"""ALS, variational fitting, block LOBPCG and block inverse iteration (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

All states live on one tree with the bond dimensions of the block; states are
lists of node tensors (legs [parent, children..., p]).  Every routine follows
the paper's algorithm in its order; where the paper leaves a choice open, the
reading taken is stated at the routine:

* ``als_solve``   -- ALS for (H - s I) y = phi (Sec. II.C.3): node-by-node
  local solves with MINRES on (H_eff - s) y_u = b_u, b_u from the (y, phi)
  identity environments; one sweep = one depth-first Euler tour from the root,
  solving each node at its first visit; QR moves the centre along the tour.
* ``fit``         -- variational fitting of sum_i c_i O_i phi_i (Sec. II.C.2):
  with the target's centre at u, the local solution is
  sum_i c_i (O_i)_eff phi_{i,u} (identity-gauge form of the local system).
* ``lobpcg``      -- Alg. lobpcg_block with the three-term recurrence.
* ``inverse_iteration`` -- Alg. block_inverse_iteration with clusters.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import mlp, ttn
from .linalg import minres, rayleigh_ritz


# ------------------------------------------------------------- env bookkeeping

class EnvCache:
    """Environments E_{u->v} of one (bra, op, ket) triple, kept valid for
    edges pointing toward the current orthogonality centre."""

    def __init__(self, tree, bra, W, ket, centre):
        self.tree, self.bra, self.W, self.ket = tree, bra, W, ket
        self.E: Dict[Tuple[int, int], np.ndarray] = ttn.all_envs_toward(tree, centre, bra, W, ket)

    def incoming(self, u) -> Dict[int, np.ndarray]:
        return {c: self.E[(c, u)] for c in ttn.nbrs(self.tree, u)}

    def update(self, u, v) -> None:
        """Recompute E_{u->v} (after node u's tensors changed, centre -> v)."""
        ein = {c: self.E[(c, u)] for c in ttn.nbrs(self.tree, u) if c != v}
        self.E[(u, v)] = ttn.env_update(self.tree, u, v, self.bra[u],
                                        None if self.W is None else self.W[u], self.ket[u], ein)


# ------------------------------------------------------------- ALS

@dataclasses.dataclass
class SolveStats:
    iters: List[int] = dataclasses.field(default_factory=list)
    resid: List[float] = dataclasses.field(default_factory=list)


def als_solve(tree, W, shift: float, phi, y0, sweeps: int, maxiter: int, rtol: float,
              stats: Optional[SolveStats] = None, local="minres"):
    """Approximate y with (H - shift) y = phi (Sec. II.C.3, Fig. als).

    local: the local map -- "minres" (the paper's), "diag" (y = b / (diag(H_eff)
    - s)), or ("learned", params) for the learned map of ``oracle.mlp``;
    "minres+diag" or ("minres+learned", params): MINRES from a start corrected
    by ``start_correction`` (not in the paper)."""
    root = tree.root
    y = ttn.canonicalize(tree, y0, root)
    phi_c = phi
    Hc = EnvCache(tree, y, W, y, root)
    Rc = EnvCache(tree, y, None, phi_c, root)
    tour = ttn.euler_tour(tree)
    for _ in range(sweeps):
        seen = set()
        for t, u in enumerate(tour):
            if u not in seen:
                seen.add(u)
                b = ttn.heff_apply(tree, u, None, phi_c[u], Rc.incoming(u))
                Hin = Hc.incoming(u)
                Wu = W[u]
                kind = local if isinstance(local, str) else local[0]
                if kind in ("minres", "minres+diag", "minres+learned"):
                    A = lambda v: ttn.heff_apply(tree, u, Wu, v, Hin, shift)
                    x0 = y[u]
                    if kind != "minres":
                        dg = ttn.heff_diag(tree, u, Wu, Hin, shift)
                        x0 = x0 + start_correction(A, b - A(x0), dg, None if kind == "minres+diag" else local[1])
                    x, it, res = minres(A, b, x0, rtol, maxiter)
                    if stats is not None:
                        stats.iters.append(it)
                        stats.resid.append(res)
                else:
                    dg = ttn.heff_diag(tree, u, Wu, Hin, shift)
                    if local == "diag":
                        x = b / dg
                    else:
                        shp = b.shape
                        A = lambda v: ttn.heff_apply(tree, u, Wu, v.reshape(shp), Hin, shift).ravel()
                        x, _ = mlp.learned_local(local[1], A, b.ravel(), dg.ravel())
                        x = x.reshape(shp)
                y[u] = x
            if t + 1 < len(tour):
                v = tour[t + 1]
                ttn.move_centre(tree, y, u, v)
                Hc.update(u, v)
                Rc.update(u, v)
    return y


def start_correction(apply_A, r0: np.ndarray, d: np.ndarray, params=None) -> np.ndarray:
    """Correction c of a MINRES start y0 for A y = b, from r0 = b - A y0 and
    the diagonal d of A (an extension, not in the paper).  params None: the
    DIAG step r0 / d at its minimal-residual scale a = <A(r0/d), r0> /
    |A(r0/d)|^2 (a = 1 where that image vanishes); otherwise the learned local
    map of ``oracle.mlp`` applied to the system A c = r0."""
    if params is None:
        g = r0 / d
        Ag = apply_A(g)
        gg = float(np.vdot(Ag, Ag))
        return (float(np.vdot(Ag, r0)) / gg if gg > 0 else 1.0) * g
    shp = r0.shape
    c, _ = mlp.learned_local(params, lambda v: apply_A(v.reshape(shp)).ravel(), r0.ravel(), d.ravel())
    return c.reshape(shp)


# ------------------------------------------------------------- fitting

def fit(tree, sources: Sequence[Tuple[float, Optional[list], list]], init, sweeps: int = 2):
    """Variational fitting of sum_i c_i O_i phi_i (O_i a TTNO or None for the
    identity) into a state with init's bond dimensions (Sec. II.C.2)."""
    root = tree.root
    y = ttn.canonicalize(tree, init, root)
    caches = [EnvCache(tree, y, Wi, phi, root) for (_, Wi, phi) in sources]
    tour = ttn.euler_tour(tree)
    for _ in range(sweeps):
        seen = set()
        for t, u in enumerate(tour):
            if u not in seen:
                seen.add(u)
                acc = np.zeros_like(y[u])
                for (c, Wi, phi), cache in zip(sources, caches):
                    acc = acc + c * ttn.heff_apply(tree, u, None if Wi is None else Wi[u], phi[u], cache.incoming(u))
                y[u] = acc
            if t + 1 < len(tour):
                v = tour[t + 1]
                ttn.move_centre(tree, y, u, v)
                for cache in caches:
                    cache.update(u, v)
    return y


def normalized(tree, state):
    st = ttn.canonicalize(tree, state, tree.root)
    nrm = ttn.norm_centre(st, tree.root)
    st[tree.root] = st[tree.root] / nrm
    return st


# ------------------------------------------------------------- LOBPCG

@dataclasses.dataclass
class LobpcgOptions:
    n_iter: int = 5
    shift: float = 0.0                # preconditioner shift s (same for all states)
    als_sweeps: int = 2
    minres_maxiter: int = 10
    minres_rtol: float = 1e-6
    fit_sweeps: int = 2
    drop_tol: float = 1e-12
    resid_tol: Optional[float] = None  # stop when every ||r_j|| <= tol (cm^-1)


def rayleigh_quotients(tree, W, xs) -> np.ndarray:
    return np.array([ttn.expectation(tree, x, W, x) / ttn.expectation(tree, x, None, x) for x in xs])


def lobpcg(tree, W, x0, opts: LobpcgOptions, history: Optional[list] = None):
    """Block LOBPCG (Alg. lobpcg_block) for the lowest len(x0) states.

    Per iteration: lambda_j = Rayleigh quotients; r_j = H x_j - lambda_j x_j
    by fitting; w_j = preconditioned residual by ALS on (H - s) w = r_j;
    subspace {x, w, p} ({x, w} on the first iteration); Gram matrices;
    Rayleigh-Ritz; p_j = sum over the w and p parts, x_j = sum over all parts,
    each fitted to the block's bond dimensions and normalised.
    """
    k = len(x0)
    xs = [normalized(tree, x) for x in x0]
    lam = rayleigh_quotients(tree, W, xs)
    ps: List = []
    for it in range(opts.n_iter):
        ws, rn = [], []
        for j in range(k):
            r = fit(tree, [(1.0, W, xs[j]), (-lam[j], None, xs[j])], xs[j], opts.fit_sweeps)
            rn.append(ttn.norm_centre(r, tree.root))
            w = als_solve(tree, W, opts.shift, r, r, opts.als_sweeps, opts.minres_maxiter, opts.minres_rtol)
            ws.append(normalized(tree, w))
        if history is not None:
            history.append({"iter": it, "lam": lam.copy(), "resid": np.array(rn)})
        if opts.resid_tol is not None and max(rn) <= opts.resid_tol:
            break
        basis = xs + ws + ps
        Ht, St = ttn.gram(tree, basis, W)
        theta, V, _ = rayleigh_ritz(Ht, St, k, opts.drop_tol)
        new_x, new_p = [], []
        for j in range(k):
            src_p = [(V[l, j], None, basis[l]) for l in range(k, len(basis))]
            src_x = [(V[l, j], None, basis[l]) for l in range(len(basis))]
            new_p.append(normalized(tree, fit(tree, src_p, basis[k + j], opts.fit_sweeps)))
            new_x.append(normalized(tree, fit(tree, src_x, xs[j], opts.fit_sweeps)))
        xs, ps = new_x, new_p
        lam = rayleigh_quotients(tree, W, xs)
    return xs, lam


# ------------------------------------------------------------- inverse iteration

def clusters_of(lam: np.ndarray, gap: float = 5.0) -> List[List[int]]:
    """Single-linkage clusters of the sorted values: a new cluster starts
    wherever consecutive values differ by >= gap (Sec. III.B)."""
    order = list(np.argsort(lam))
    out = [[order[0]]]
    for a, b in zip(order[:-1], order[1:]):
        if lam[b] - lam[a] >= gap:
            out.append([b])
        else:
            out[-1].append(b)
    return out


@dataclasses.dataclass
class IIOptions:
    n_iter: int = 5
    sweeps: int = 1
    minres_maxiter: int = 10000
    minres_rtol: float = 1e-10
    fit_sweeps: int = 2
    gap: float = 5.0
    drop_tol: float = 1e-12
    dlam_tol: Optional[float] = None  # stop when every |d lambda| < tol
    # Optional safeguard, NOT part of Alg. block_inverse_iteration (off by
    # default): keep a cluster's previous states when its update raised a
    # Rayleigh quotient by more than mono_tol (cm^-1).
    monotone: bool = False
    mono_tol: float = 1e-7


def inverse_iteration(tree, W, xs, lam, opts: IIOptions, history: Optional[list] = None):
    """Block inverse iteration (Alg. block_inverse_iteration), clusters fixed
    from the input Rayleigh quotients, shift = cluster mean, followed by one
    global Rayleigh-Ritz over all states.  Returns (states, Ritz values).

    Per outer iteration and cluster: s = mean Rayleigh quotient of the
    cluster; each state is replaced by its normalised ALS solution of
    (H - s) y = x_j; a cluster of more than one state is then orthogonalised
    by its own Rayleigh-Ritz problem (x_j <- sum_k V[k, j] x_k, fitted), and
    the Rayleigh quotients are recomputed.

    opts.monotone (off by default; a safeguard that is not in the paper): at
    a fixed bond dimension the ALS solve of a nearly singular shifted system
    can move a state away from its eigenvector; with the option on, a cluster
    whose update raised any Rayleigh quotient by more than mono_tol keeps its
    previous states."""
    xs = [normalized(tree, x) for x in xs]
    lam = np.array(lam, dtype=np.float64)
    cl = clusters_of(lam, opts.gap)
    for it in range(opts.n_iter):
        old = lam.copy()
        for c in cl:
            prev = {j: xs[j] for j in c}
            s = float(np.mean(lam[c]))
            for j in c:
                y = als_solve(tree, W, s, xs[j], xs[j], opts.sweeps, opts.minres_maxiter, opts.minres_rtol)
                xs[j] = normalized(tree, y)
            if len(c) > 1:
                sub = [xs[j] for j in c]
                Ht, St = ttn.gram(tree, sub, W)
                th, V, _ = rayleigh_ritz(Ht, St, len(c), opts.drop_tol)
                newx = []
                for jj in range(len(c)):
                    src = [(V[l, jj], None, sub[l]) for l in range(len(c))]
                    newx.append(normalized(tree, fit(tree, src, sub[jj], opts.fit_sweeps)))
                for jj, j in enumerate(c):
                    xs[j] = newx[jj]
            for j in c:
                lam[j] = ttn.expectation(tree, xs[j], W, xs[j])
            if opts.monotone and max(lam[j] - old[j] for j in c) > opts.mono_tol:
                for j in c:
                    xs[j] = prev[j]
                    lam[j] = old[j]
        if history is not None:
            history.append({"iter": it, "lam": lam.copy()})
        if opts.dlam_tol is not None and np.max(np.abs(lam - old)) < opts.dlam_tol:
            break
    Ht, St = ttn.gram(tree, xs, W)
    theta, _, _ = rayleigh_ritz(Ht, St, len(xs), opts.drop_tol)
    return xs, theta
