"""Block LOBPCG and block inverse iteration on the GPU path.

Host-side control only: every tensor operation (environment updates, H_eff
products, MINRES, QR gauge moves, fitting sums, Gram closures, Rayleigh-Ritz,
normalisation, norms, coefficient gathers, precision promotion) runs in
libttn's HIP kernels through the C ABI.  The host reads back scalars (Rayleigh
quotients, residual norms) to decide clusters and stopping; PyTorch provides
device buffers (allocated once per solver) and plain copies between them.

Algorithms: Alg. lobpcg_block with the three-term recurrence (Eq. lobpcg
update) and Alg. block_inverse_iteration, read as: the subspace {x, w} on
the first iteration, x_j a combination of all 3n basis states, clusters
fixed after LOBPCG, and a final global Rayleigh-Ritz.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import ttn


@dataclasses.dataclass
class LobpcgOpts:
    n_iter: int = 5
    shift: Optional[float] = None     # preconditioner shift; None -> min RQ(x0) - 837 cm^-1
    als_sweeps: int = 2
    minres_maxiter: int = 10
    minres_rtol: float = 1e-6
    fit_sweeps: int = 2
    drop_tol: float = 1e-12
    resid_tol: Optional[float] = None
    precond: str = "minres"           # local map of the ALS preconditioner: "minres", "diag", "learned", or
                                      # "minres+diag" / "minres+learned" (MINRES from a corrected start)
    mlp: Optional[torch.Tensor] = None  # learned map parameters (device FP32)
    mlp_compute: int = ttn.BF16
    residual: str = "fit"             # H x_j by variational fitting ("fit") or successive randomized
                                      # compression with sketch size D ("src", Sec. II.C.1)
    src_seed: int = 1234              # seed of the SRC test matrices (one draw per iteration)


@dataclasses.dataclass
class IIOpts:
    n_iter: int = 5
    sweeps: int = 1
    minres_maxiter: int = 10000
    minres_rtol: float = 1e-10
    fit_sweeps: int = 2
    gap: float = 5.0
    drop_tol: float = 1e-12
    dlam_tol: Optional[float] = None
    # optional safeguard, not part of Alg. block_inverse_iteration (off by default): a cluster whose
    # update raised a Rayleigh quotient by more than mono_tol (cm^-1) keeps its previous states
    monotone: bool = False
    mono_tol: float = 1e-7
    refine: int = 0         # > 0: local solves by FP64 refinement around FP32-arithmetic MINRES (FP64 solver)
    # SPD preconditioning of the local MINRES (not in the paper): "none", "diag" (D = |diag(H_eff) - s|) or
    # "damped" (D = sqrt((diag - s)^2 + gamma^2), gamma = precond_damp * rms(diag - s): the learned damping)
    precond: str = "none"
    precond_damp: float = 0.1


def post_order_edges(tree: ttn.Tree):
    """Edges u -> parent(u) with every child before its parent."""
    out = []

    def rec(u):
        for c in tree.children[u]:
            rec(c)
        if tree.parent[u] >= 0:
            out.append((u, tree.parent[u]))

    rec(tree.root)
    return out


def build_ttno(gt: ttn.Tree, tree, model):
    """Site tensors and operator bonds of the model's TTNO (library host compiler)."""
    return ttn.sop_build(gt, tree.mode, model.omega, model.dims, model.monomials, model.coefs)


class TTNEigensolver:
    """GPU block eigensolver for one Hamiltonian on one tree.

    tree: workloads.Tree; model: workloads.SOPModel; the initial block comes
    as [state][node] host arrays (seeded input, not yet canonical).
    precision: "fp64" (plain) or "fp32" / "bf16" (contractions in FP32 / BF16
    matrix cores, FP32 storage; Rayleigh-Ritz always FP64), or "f64_f32" (the
    mixed form: FP64 storage, every contraction with the Hamiltonian that
    builds the block -- the H~ Gram environments, the residual fits, the
    preconditioner's sweeps and fits -- on FP32 matrix cores, while the
    overlap S~, the Rayleigh quotients and Rayleigh-Ritz stay in FP64
    arithmetic).
    """

    def __init__(self, ctx: ttn.Context, tree, model, D: int, k: int, precision: str = "fp64",
                 workspace_pairs: int = 4096, graphs: bool = False, ttno=None,
                 env_budget_bytes: Optional[int] = None, pre_compute: Optional[int] = None):
        import workloads as wl
        self.ctx, self.k = ctx, k
        self.graphs = graphs  # replay the sweeps as HIP graphs (needs a non-null context stream)
        self.wtree = tree
        self.gt = ttn.Tree(tree.parent, tree.phys)
        # the host compiler's TTNO (or a prebuilt one: (site tensors, operator bonds))
        W, M = ttno if ttno is not None else build_ttno(self.gt, tree, model)
        self.M = [max(1, m) for m in M]
        self._model, self._precision, self._ttno_host, self._pre_compute = model, precision, (W, M), pre_compute
        self.sdt = ttn.F64 if precision in ("fp64", "f64_f32") else ttn.F32
        # bulk compute type, and the one of the exact quantities (S~, Rayleigh quotients)
        self.compute = {"fp64": ttn.F64, "fp32": ttn.F32, "bf16": ttn.BF16, "f64_f32": ttn.F64_F32}[precision]
        self.compute_exact = ttn.F64 if self.sdt == ttn.F64 else self.compute
        self.tdt = ttn.torch_dtype(self.sdt)
        self.Wd = [torch.from_numpy(np.ascontiguousarray(w)).to(device="cuda", dtype=self.tdt) for w in W]
        self.op = ttn.TTNO(ctx, self.gt, self.Wd, self.M, self.sdt)
        self.bonds = [max(1, b) for b in wl.bond_dims(tree, D)]
        self.zpe = model.zpe_harmonic
        n = tree.n
        self.root = tree.root
        self.B = ttn.Block(ctx, self.gt, 3 * k, self.bonds, self.sdt)     # basis [x | w | p]
        self.R = ttn.Block(ctx, self.gt, k, self.bonds, self.sdt)         # residuals
        self.Wp = ttn.Block(ctx, self.gt, k, self.bonds, self.sdt)        # preconditioned residuals
        self.XN = ttn.Block(ctx, self.gt, k, self.bonds, self.sdt)        # recombined x
        self.PN = ttn.Block(ctx, self.gt, k, self.bonds, self.sdt)        # recombined p
        self.Y = ttn.Block(ctx, self.gt, k, self.bonds, self.sdt)         # inverse-iteration target
        self.up_edges = post_order_edges(self.gt)
        # Gram environments are kept for pair_cap pairs at a time; a byte
        # budget caps it (bigger chunks: fewer, fuller launches)
        es = 8 if self.sdt == ttn.F64 else 4
        per_pair = es * sum(self.bonds[u] * (self.M[u] + 1) * self.bonds[u] for (u, _) in post_order_edges(self.gt))
        self.pair_cap = workspace_pairs
        if env_budget_bytes is not None:
            self.pair_cap = int(max(16, min(workspace_pairs, env_budget_bytes // max(per_pair, 1))))
        dev = "cuda"
        up_slots = [2 * u for (u, _) in self.up_edges]
        self.genv_H = ttn.Envs(ctx, self.gt, self.pair_cap, self.bonds, self.M, self.bonds, self.sdt, edges=up_slots)
        self.genv_I = ttn.Envs(ctx, self.gt, self.pair_cap, self.bonds, None, self.bonds, self.sdt, edges=up_slots)
        self.norms = torch.zeros(3 * k, dtype=torch.float64, device=dev)
        # residual fit: r_j = H x_j - lambda_j x_j
        self.lam_d = torch.zeros(k, dtype=torch.float64, device=dev)
        self.neglam_d = torch.zeros(k, dtype=torch.float64, device=dev)
        ones = torch.ones(k, dtype=torch.float64, device=dev)
        self._ones = ones
        idx = list(range(k))
        self.sw_res = ttn.Sweep(ctx, self.gt, None, self.R,
                                [(self.op, self.B, idx, idx, ones), (None, self.B, idx, idx, self.neglam_d)],
                                compute=self.compute)
        self.shift_d = torch.zeros(k, dtype=torch.float64, device=dev)
        # the preconditioner's ALS only shapes the search directions: it may run
        # on FP32 matrix cores over the FP64 tensors (pre_compute=F64_F32)
        self.sw_pre = ttn.Sweep(ctx, self.gt, self.op, self.Wp, [(None, self.R, idx, idx, None)], shift=self.shift_d,
                                compute=self.compute if pre_compute is None else pre_compute)
        # recombination fits: x_j = sum_l V[l, j] B_l ; p_j = sum_{l >= k} V[l, j] B_l
        m3 = 3 * k
        self.cx_t = [j for j in range(k) for l in range(m3)]
        self.cx_s = [l for j in range(k) for l in range(m3)]
        self.cp_t = [j for j in range(k) for l in range(k, m3)]
        self.cp_s = [l for j in range(k) for l in range(k, m3)]
        self.cx_d = torch.zeros(len(self.cx_t), dtype=torch.float64, device=dev)
        self.cp_d = torch.zeros(len(self.cp_t), dtype=torch.float64, device=dev)
        self.sw_x = ttn.Sweep(ctx, self.gt, None, self.XN, [(None, self.B, self.cx_t, self.cx_s, self.cx_d)],
                              compute=self.compute)
        self.sw_p = ttn.Sweep(ctx, self.gt, None, self.PN, [(None, self.B, self.cp_t, self.cp_s, self.cp_d)],
                              compute=self.compute)
        self.ix_gather = torch.tensor([l * k + j for j, l in zip(self.cx_t, self.cx_s)], dtype=torch.int32, device=dev)
        self.ip_gather = torch.tensor([l * k + j for j, l in zip(self.cp_t, self.cp_s)], dtype=torch.int32, device=dev)
        self.rn2 = torch.zeros(k, dtype=torch.float64, device=dev)   # squared residual norms
        self.rn = torch.zeros(k, dtype=torch.float64, device=dev)    # residual norms
        ld = 3 * k
        self.GH = torch.zeros(ld * ld, dtype=torch.float64, device=dev)  # Gram matrices (row-major ld x ld)
        self.GS = torch.zeros(ld * ld, dtype=torch.float64, device=dev)
        self._pairs = {}  # device pair / scatter tables and closure outputs, by pair-list name
        self.history: List[dict] = []
        self._sw_ii = None
        self.cluster_rr_calls = 0  # in-cluster Rayleigh-Ritz steps of inverse iteration (clusters of > 1 state)
        self._cl_tables = None     # device tables of the in-cluster Rayleigh-Ritz (clusters are fixed)
        self._src = None           # successive randomized compression of H x (created on first use)

    # ------------------------------------------------------------ block plumbing

    def _copy_rows(self, dst: ttn.Block, d0: int, src: ttn.Block, s0: int, cnt: int):
        for u in range(self.gt.n):
            dst.t[u][d0:d0 + cnt].copy_(src.t[u][s0:s0 + cnt])

    def load_block(self, states):
        """Upload host states into rows [0, k) of the basis, canonicalise at
        the root (QR moves on the device) and normalise."""
        k = self.k
        for u in range(self.gt.n):
            arr = np.stack([states[j][u] for j in range(k)])
            self.B.t[u][:k].copy_(torch.from_numpy(arr).to(self.tdt))
            self.B.t[u][k:].zero_()
        self._canonicalize(self.B)
        ttn.block_normalize_node(self.ctx, self.B, self.root, self.norms)

    def _canonicalize(self, blk: ttn.Block):
        for (u, p) in self.up_edges:
            ttn.block_move_centre(self.ctx, blk, u, p)

    # ------------------------------------------------------------ Gram / Rayleigh quotients

    def _pair_set(self, name, pairs_a: List[int], pairs_b: List[int], la=None, lb=None):
        """Device tables of a pair list (chunked to the environment capacity),
        its closure outputs and, with la / lb, its symmetric scatter indices;
        built once per name."""
        ps = self._pairs.get(name)
        if ps is None or ps["n"] != len(pairs_a) or ps["key"] != (tuple(pairs_a), tuple(pairs_b)):
            n = len(pairs_a)
            i32 = dict(dtype=torch.int32, device="cuda")
            ps = {"n": n, "key": (tuple(pairs_a), tuple(pairs_b)),
                  "chunks": [(c0, min(n, c0 + self.pair_cap),
                              torch.tensor(pairs_a[c0:c0 + self.pair_cap], **i32),
                              torch.tensor(pairs_b[c0:c0 + self.pair_cap], **i32))
                             for c0 in range(0, n, self.pair_cap)],
                  "H": torch.zeros(n, dtype=torch.float64, device="cuda"),
                  "S": torch.zeros(n, dtype=torch.float64, device="cuda")}
            if la is not None:
                ps["la"] = torch.tensor(la, **i32)
                ps["lb"] = torch.tensor(lb, **i32)
            self._pairs[name] = ps
        return ps

    def gram(self, blk: ttn.Block, pairs_a: List[int], pairs_b: List[int], with_H=True, with_S=True, name=None,
             exact_H=False):
        """Closures <a|H|b> and <a|b> for the listed pairs (device double arrays).
        <a|H|b> in the bulk compute type unless exact_H; <a|b> in the exact one."""
        ps = self._pair_set(name or ("pairs", len(pairs_a)), pairs_a, pairs_b)
        outH, outS = ps["H"], ps["S"]
        cH = self.compute_exact if exact_H else self.compute
        for (c0, c1, pa, pb) in ps["chunks"]:
            for (op, env, out, comp) in ((self.op, self.genv_H, outH, cH), (None, self.genv_I, outS,
                                                                            self.compute_exact)):
                if (op is not None and not with_H) or (op is None and not with_S):
                    continue
                for (u, p) in self.up_edges:
                    ttn.ttno_env_update(self.ctx, self.gt, op, blk, blk, pa, pb, u, p, env, comp)
                ttn.ttno_env_close(self.ctx, self.gt, op, blk, blk, pa, pb, self.root, env, out[c0:c1],
                                   comp)
        return outH, outS

    def rayleigh_quotients(self, blk: ttn.Block, rows: List[int]) -> torch.Tensor:
        H, _ = self.gram(blk, rows, rows, with_S=False, name=("rq", len(rows)), exact_H=True)
        return H  # states are normalised

    def _gram_matrices(self, blk: ttn.Block, name, rows_a: List[int], rows_b: List[int], la: List[int],
                       lb: List[int], size: int, exact_H: bool = False):
        """Gram closures of the listed pairs scattered symmetrically into the
        preallocated H~ / S~ buffers (entries la / lb; only the problems'
        m x m blocks are read by Rayleigh-Ritz)."""
        ps = self._pair_set(name, rows_a, rows_b, la, lb)
        hv, sv = self.gram(blk, rows_a, rows_b, name=name, exact_H=exact_H)
        Hm, Sm = self.GH[:size], self.GS[:size]
        ttn.scatter_sym(self.ctx, ps["la"], ps["lb"], hv, Hm)
        ttn.scatter_sym(self.ctx, ps["la"], ps["lb"], sv, Sm)
        return Hm, Sm

    # ------------------------------------------------------------ LOBPCG

    def lobpcg_start(self, opts: LobpcgOpts):
        """Rayleigh quotients of the loaded block and the preconditioner shift."""
        k = self.k
        self._opts = opts
        self._t0 = time.perf_counter()
        lam = self.rayleigh_quotients(self.B, list(range(k)))
        self.lam_d.copy_(lam)
        s = float(lam.min().item()) - 837.0 if opts.shift is None else opts.shift
        self.shift_d.fill_(s)
        self._have_p = False
        self._it = 0

    def lobpcg_step(self, log=None) -> bool:
        """One block-LOBPCG iteration; returns False when the residual
        criterion stopped the iteration before the subspace update."""
        ctx, k, root, opts = self.ctx, self.k, self.root, self._opts
        it = self._it
        self._it += 1
        # residual r_j = H x_j - lambda_j x_j by fitting, or H x_j by SRC then
        # r_j = y_j - lambda_j x_j by an identity fit
        ttn.vec_scale(ctx, self.lam_d, -1.0, self.neglam_d)
        self._copy_rows(self.R, 0, self.B, 0, k)
        if opts.residual == "src":
            self._src_residual(opts)
        else:
            self.sw_res.run(ttn.SOLVE_FIT, opts.fit_sweeps, init=True, graph=self.graphs)
        ttn.block_node_norms2(ctx, self.R, root, self.rn2)
        ttn.vec_sqrt(ctx, self.rn2, self.rn)
        # preconditioned residual: (H - s) w = r by ALS
        self._copy_rows(self.Wp, 0, self.R, 0, k)
        mode, warm = {"minres": (ttn.SOLVE_MINRES, ttn.WARM_NONE), "diag": (ttn.SOLVE_DIAG, ttn.WARM_NONE),
                      "learned": (ttn.SOLVE_LEARNED, ttn.WARM_NONE),
                      "minres+diag": (ttn.SOLVE_MINRES, ttn.WARM_DIAG),
                      "minres+learned": (ttn.SOLVE_MINRES, ttn.WARM_LEARNED)}[opts.precond]
        self.sw_pre.run(mode, opts.als_sweeps, init=True, graph=self.graphs, maxiter=opts.minres_maxiter,
                        rtol=opts.minres_rtol, mlp=opts.mlp, mlp_compute=opts.mlp_compute, warm=warm)
        ttn.block_normalize_node(ctx, self.Wp, root)
        self._copy_rows(self.B, k, self.Wp, 0, k)
        rnorm = self.rn.cpu().numpy()
        lam_h = self.lam_d.cpu().numpy()
        rec = {"iter": it, "t": time.perf_counter() - self._t0, "lam": lam_h + self.zpe, "resid": rnorm}
        self.history.append(rec)
        if log:
            log(rec)
        if opts.resid_tol is not None and rnorm.max() <= opts.resid_tol:
            return False
        m = 3 * k if self._have_p else 2 * k
        ia, ib = [], []
        for a in range(m):
            for b in range(a, m):
                ia.append(a)
                ib.append(b)
        ld = 3 * k
        la = [a * ld + b for a, b in zip(ia, ib)]
        lb = [b * ld + a for a, b in zip(ia, ib)]
        Hm, Sm = self._gram_matrices(self.B, ("subspace", m), ia, ib, la, lb, ld * ld)
        ev, V, rank = ttn.rayleigh_ritz(ctx, Hm.view(1, ld, ld), Sm.view(1, ld, ld), [m], k, opts.drop_tol)
        Vf = V[0].reshape(-1)  # [ld][k] row-major: V[l, j] at l*k + j
        ttn.vec_gather(ctx, self.ix_gather, Vf, self.cx_d)
        ttn.vec_gather(ctx, self.ip_gather, Vf, self.cp_d)
        # p_j = sum_{l >= k} V[l, j] s_l ; x_j = sum_l V[l, j] s_l  (fitted)
        self._copy_rows(self.PN, 0, self.B, k, k)
        self.sw_p.run(ttn.SOLVE_FIT, opts.fit_sweeps, init=True, graph=self.graphs)
        self._copy_rows(self.XN, 0, self.B, 0, k)
        self.sw_x.run(ttn.SOLVE_FIT, opts.fit_sweeps, init=True, graph=self.graphs)
        ttn.block_normalize_node(ctx, self.PN, root)
        ttn.block_normalize_node(ctx, self.XN, root)
        self._copy_rows(self.B, 0, self.XN, 0, k)
        self._copy_rows(self.B, 2 * k, self.PN, 0, k)
        self._have_p = True
        lam = self.rayleigh_quotients(self.B, list(range(k)))
        self.lam_d.copy_(lam)
        return True

    def _src_residual(self, opts: LobpcgOpts):
        """y_j ~ H x_j by successive randomized compression (sketch size D),
        then r_j = y_j - lambda_j x_j fitted into the residual block."""
        k = self.k
        if self._src is None:
            D = max(self.bonds)
            self.XS = ttn.Block(self.ctx, self.gt, k, self.bonds, self.sdt)
            self.YS = ttn.Block(self.ctx, self.gt, k, [max(1, b) for b in ttn.src_bonds(self.gt, D)], self.sdt)
            sc = ttn.F64 if self.sdt == ttn.F64 else ttn.F32
            self._src = ttn.Src(self.ctx, self.gt, self.op, self.XS, self.YS, D, sc)
            self._src_chi = D
            idx = list(range(k))
            self.sw_res_src = ttn.Sweep(self.ctx, self.gt, None, self.R,
                                        [(None, self.YS, idx, idx, self._ones), (None, self.XS, idx, idx, self.neglam_d)],
                                        compute=self.compute_exact if self.sdt == ttn.F64 else self.compute)
            self._src_gen = torch.Generator(device="cuda")
            self._src_gen.manual_seed(opts.src_seed)
        self._copy_rows(self.XS, 0, self.B, 0, k)
        om = [torch.randn(self._src_chi, self.gt.phys[u], generator=self._src_gen, device="cuda", dtype=self.tdt)
              if self.gt.phys[u] > 1 else None for u in range(self.gt.n)]
        self._src.apply(om)
        self.sw_res_src.run(ttn.SOLVE_FIT, opts.fit_sweeps, init=True, graph=self.graphs)

    def harvest(self, rows_per_node: int, maxiter: int = 300, rtol: float = 1e-10, seed: int = 0):
        """Training pairs for the learned local map: one ALS sweep of plain
        MINRES solves (H - s) w = r on the current residual block (the
        preconditioner's own systems, solved to rtol), recording at each node,
        right after its solve, the tile features of (b, diag(H_eff) - s) and
        the solution tiles.  Returns device tensors X [n][128], T [n][64]
        with up to rows_per_node tile rows per node (sampled)."""
        k, root = self.k, self.root
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        self._copy_rows(self.Wp, 0, self.R, 0, k)
        self.sw_pre.init(root)
        xs, ts = [], []

        def on_solved(u):
            n = int(np.prod(self.Wp.legdims(u)))
            nt = -(-n // 64)
            X = torch.empty(k * nt, 128, dtype=torch.float32, device="cuda")
            T = torch.empty(k * nt, 64, dtype=torch.float32, device="cuda")
            sc = torch.empty(k, 2, dtype=torch.float64, device="cuda")
            self.sw_pre.harvest(u, X, T, sc)
            sel = torch.randperm(k * nt, generator=g)[:rows_per_node].to("cuda")
            xs.append(X[sel])
            ts.append(T[sel])

        ttn.run_sweep(self.sw_pre, self.gt, ttn.SOLVE_MINRES, maxiter, rtol, on_solved=on_solved)
        return torch.cat(xs), torch.cat(ts)

    def lobpcg(self, opts: LobpcgOpts, log=None):
        self.lobpcg_start(opts)
        for _ in range(opts.n_iter):
            if not self.lobpcg_step(log):
                break
        return self.lam_d.cpu().numpy() + self.zpe

    # ------------------------------------------------------------ bond growth

    def grow(self, D: int, n_sketch: Optional[int] = None, omegas=None, seed: int = 0) -> "TTNEigensolver":
        """A solver at the larger bond dimension D holding this solver's k
        states grown by the residual-driven expansion (ttn_expand: the current
        bases kept, each bond's new directions from a rank-revealing QR of the
        local residual of H x), with the same Rayleigh quotients, shift and
        options; the LOBPCG search directions are not carried over.  omegas:
        host [d_u x n_sketch] sketch matrices per node (None at auxiliary
        nodes), else drawn on the device from `seed`."""
        ctx, k = self.ctx, self.k
        hi = TTNEigensolver(ctx, self.wtree, self._model, D, k, self._precision, graphs=self.graphs,
                            ttno=self._ttno_host, pre_compute=self._pre_compute)
        growth = max(h - l for u, (h, l) in enumerate(zip(hi.bonds, self.bonds)) if u != self.root)
        n = n_sketch if n_sketch is not None else max(1, growth)
        XS = ttn.Block(ctx, self.gt, k, self.bonds, self.sdt)
        YS = ttn.Block(ctx, self.gt, k, hi.bonds, self.sdt)
        self._copy_rows(XS, 0, self.B, 0, k)
        if omegas is None:
            gen = torch.Generator(device="cuda")
            gen.manual_seed(seed)
            om = [torch.randn(n, self.gt.phys[u], generator=gen, device="cuda", dtype=self.tdt)
                  if self.gt.phys[u] > 1 else None for u in range(self.gt.n)]
        else:
            om = [torch.from_numpy(np.ascontiguousarray(np.asarray(o).T)).to(device="cuda", dtype=self.tdt)
                  if o is not None else None for u, o in enumerate(omegas)]
        ex = ttn.Expand(ctx, self.gt, self.op, XS, YS, n, ttn.F64 if self.sdt == ttn.F64 else ttn.F32)
        ex.apply(om)
        for u in range(self.gt.n):
            hi.B.t[u][:k].copy_(YS.t[u])
            hi.B.t[u][k:].zero_()
        ex.close()
        hi._canonicalize(hi.B)
        ttn.block_normalize_node(ctx, hi.B, hi.root, hi.norms)
        hi.lam_d.copy_(hi.rayleigh_quotients(hi.B, list(range(k))))
        hi.shift_d.copy_(self.shift_d)
        hi._opts = getattr(self, "_opts", None)
        hi._have_p = False
        hi._it = getattr(self, "_it", 0)
        hi._t0 = getattr(self, "_t0", time.perf_counter())
        return hi

    # ------------------------------------------------------------ inverse iteration

    @staticmethod
    def clusters_of(lam: np.ndarray, gap: float):
        order = list(np.argsort(lam))
        out = [[order[0]]]
        for a, b in zip(order[:-1], order[1:]):
            if lam[b] - lam[a] >= gap:
                out.append([b])
            else:
                out[-1].append(b)
        return out

    def inverse_iteration(self, opts: IIOpts, log=None):
        ctx, k, root = self.ctx, self.k, self.root
        t_start = time.perf_counter()
        lam = self.lam_d.cpu().numpy().copy()
        cl = self.clusters_of(lam, opts.gap)
        idx = list(range(k))
        if self._sw_ii is None:
            # target Y, source x (rows [0, k) of the basis)
            # inverse iteration is the refinement: its solves and recombination in the exact type
            self._sw_ii = ttn.Sweep(ctx, self.gt, self.op, self.Y, [(None, self.B, idx, idx, None)],
                                    shift=self.shift_d, compute=self.compute_exact)
            # recombination inside clusters: x_j = sum_{l in c(j)} V_c[l, j] x_l
            self.ci_t = [j for c in cl for j in c for l in c]
            self.ci_s = [l for c in cl for j in c for l in c]
            self.ci_d = torch.zeros(len(self.ci_t), dtype=torch.float64, device="cuda")
            self._sw_rec = ttn.Sweep(ctx, self.gt, None, self.XN, [(None, self.B, self.ci_t, self.ci_s, self.ci_d)],
                                     compute=self.compute_exact)
            self._clusters = cl
        cl = self._clusters
        big = [c for c in cl if len(c) > 1]
        for it in range(opts.n_iter):
            old = lam.copy()
            shifts = np.zeros(k)
            for c in cl:
                shifts[c] = float(np.mean(lam[c]))
            self.shift_d.copy_(torch.from_numpy(shifts))
            if opts.monotone:
                self._copy_rows(self.B, k, self.B, 0, k)  # previous states (basis rows k..2k are free here)
            self._copy_rows(self.Y, 0, self.B, 0, k)
            self._sw_ii.init(root)
            col = []
            for _ in range(opts.sweeps):
                ttn.run_sweep(self._sw_ii, self.gt, ttn.SOLVE_MINRES, opts.minres_maxiter, opts.minres_rtol,
                              collect=col, refine=opts.refine,
                              precond={"none": ttn.PRECOND_NONE, "diag": ttn.PRECOND_DIAG,
                                       "damped": ttn.PRECOND_DAMPED_DIAG}[opts.precond],
                              precond_damp=opts.precond_damp)
            ttn.block_normalize_node(ctx, self.Y, root)
            self._copy_rows(self.B, 0, self.Y, 0, k)
            if big:
                self._cluster_rr(big, opts)
            lam = self.rayleigh_quotients(self.B, idx).cpu().numpy()
            reverted = []
            if opts.monotone:
                for c in cl:
                    if max(lam[j] - old[j] for j in c) > opts.mono_tol:
                        for j in c:
                            self._copy_rows(self.B, j, self.B, k + j, 1)
                            lam[j] = old[j]
                        reverted += list(c)
            self.lam_d.copy_(torch.from_numpy(lam))
            rec = {"iter": it, "t": time.perf_counter() - t_start, "lam": lam + self.zpe, "reverted": reverted,
                   "minres_iters": {int(u): int(t.max().item()) for u, t in col},
                   "minres_iters_total": [int(x) for x in sum(t.cpu() for _, t in col).tolist()] if col else []}
            self.history.append(rec)
            if log:
                log(rec)
            if opts.dlam_tol is not None and np.max(np.abs(lam - old)) < opts.dlam_tol:
                break
        return self.final_rr(opts.drop_tol)

    def _cluster_rr(self, big, opts: IIOpts):
        ctx, k, root = self.ctx, self.k, self.root
        self.cluster_rr_calls += 1
        ld = max(len(c) for c in big)
        if self._cl_tables is None:
            ia, ib, la, lb = [], [], [], []
            for ci, c in enumerate(big):
                for a in range(len(c)):
                    for b in range(a, len(c)):
                        ia.append(c[a])
                        ib.append(c[b])
                        la.append(ci * ld * ld + a * ld + b)
                        lb.append(ci * ld * ld + b * ld + a)
            # recombination coefficients in the fitting sweep's term order:
            # V[c][l, j] for the members of a cluster, 1 for a singleton
            big_index = {tuple(c): i for i, c in enumerate(big)}
            gidx = []
            for c in self._clusters:
                if len(c) == 1:
                    gidx.append(-1)
                    continue
                ci = big_index[tuple(c)]
                for jj in range(len(c)):
                    for ll in range(len(c)):
                        gidx.append(ci * ld * ld + ll * ld + jj)
            self._cl_tables = (ia, ib, la, lb, torch.tensor(gidx, dtype=torch.int32, device="cuda"))
        ia, ib, la, lb, gidx = self._cl_tables
        Hm, Sm = self._gram_matrices(self.B, "clusters", ia, ib, la, lb, len(big) * ld * ld, exact_H=True)
        ev, V, rank = ttn.rayleigh_ritz(ctx, Hm.view(len(big), ld, ld), Sm.view(len(big), ld, ld),
                                        [len(c) for c in big], ld, opts.drop_tol)
        ttn.vec_gather(ctx, gidx, V.reshape(-1), self.ci_d, fill=1.0)
        self._copy_rows(self.XN, 0, self.B, 0, k)
        self._sw_rec.run(ttn.SOLVE_FIT, opts.fit_sweeps, init=True, graph=self.graphs)
        ttn.block_normalize_node(ctx, self.XN, root)
        self._copy_rows(self.B, 0, self.XN, 0, k)

    def final_rr(self, drop_tol: float = 1e-12) -> np.ndarray:
        """One global Rayleigh-Ritz over the k states (removes the
        non-orthogonality of separately solved states)."""
        k = self.k
        ia, ib = [], []
        for a in range(k):
            for b in range(a, k):
                ia.append(a)
                ib.append(b)
        la = [a * k + b for a, b in zip(ia, ib)]
        lb = [b * k + a for a, b in zip(ia, ib)]
        Hm, Sm = self._gram_matrices(self.B, "final", ia, ib, la, lb, k * k, exact_H=True)
        ev, V, rank = ttn.rayleigh_ritz(self.ctx, Hm.view(1, k, k), Sm.view(1, k, k), [k], k, drop_tol)
        return ev[0].cpu().numpy() + self.zpe


class MixedEigensolver:
    """Mixed-precision form: block LOBPCG with FP32 storage and FP32 (or
    BF16) matrix-core contractions as the warm start, then the block is
    promoted to FP64 storage and refined.  hi = "f64_f32" (default) refines
    with the bulk H contractions still on FP32 matrix cores and the overlap
    S~, the Rayleigh quotients, Rayleigh-Ritz and the inverse-iteration
    solves in FP64; hi = "fp64" refines with every contraction in FP64."""

    def __init__(self, ctx: ttn.Context, tree, model, D: int, k: int, low: str = "fp32", ttno=None,
                 env_budget_bytes: Optional[int] = None, hi_pre_compute: Optional[int] = None,
                 hi: str = "f64_f32"):
        if ttno is None:
            ttno = build_ttno(ttn.Tree(tree.parent, tree.phys), tree, model)
        self.lo = TTNEigensolver(ctx, tree, model, D, k, precision=low, ttno=ttno, env_budget_bytes=env_budget_bytes)
        self.hi = TTNEigensolver(ctx, tree, model, D, k, precision=hi, ttno=ttno,
                                 env_budget_bytes=env_budget_bytes, pre_compute=hi_pre_compute)
        self.k = k
        self.history: List[dict] = []

    def load_block(self, states):
        self.lo.load_block(states)

    def promote(self):
        """Copy the x and p parts of the low-precision basis into the FP64
        solver (a cast, on the device) and continue from there."""
        k = self.k
        ttn.block_convert(self.hi.ctx, self.lo.B, self.hi.B, 3 * k)
        self.hi.lam_d.copy_(self.lo.lam_d)
        self.hi.shift_d.copy_(self.lo.shift_d)
        self.hi._opts = self.lo._opts
        self.hi._have_p = self.lo._have_p
        self.hi._it = self.lo._it
        self.hi._t0 = self.lo._t0
        # refresh the Rayleigh quotients in FP64
        self.hi.lam_d.copy_(self.hi.rayleigh_quotients(self.hi.B, list(range(k))))
