"""Thin ctypes binding of libttn.so (argument marshalling only).

Device memory and streams come from PyTorch; every arithmetic step runs in the
library's HIP kernels.  The binding refuses to run without the built library:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttn.so")

F64, F32, BF16, F64_F32 = 0, 1, 2, 3
HEFF_APPLY, HEFF_NO_SHIFT, HEFF_DIAG, HEFF_ACCUM = 0, 1, 2, 4
SOLVE_MINRES, SOLVE_DIAG, SOLVE_FIT, SOLVE_SKIP, SOLVE_LEARNED = 0, 1, 2, 3, 4
WARM_NONE, WARM_DIAG, WARM_LEARNED = 0, 1, 2
PRECOND_NONE, PRECOND_DIAG, PRECOND_DAMPED_DIAG = 0, 1, 2

_lib = None

# exported entry points and their ctypes signatures (all return int32 status
# unless noted)
_P = C.c_void_p
_I = C.c_int32
_PI = C.POINTER(C.c_int32)
_SIGS = {
    "ttn_ctx_create": [C.c_int, _P, C.c_size_t, C.POINTER(_P)],
    "ttn_ctx_set_stream": [_P, _P],
    "ttn_ctx_sync": [_P],
    "ttn_ctx_destroy": [_P],
    "ttn_tree_create": [_I, _PI, _PI, C.POINTER(_P)],
    "ttn_tree_destroy": [_P],
    "ttn_ttno_create": [_P, _P, _PI, C.c_int, C.POINTER(_P), C.POINTER(_P)],
    "ttn_ttno_destroy": [_P],
    "ttn_block_create": [_P, _P, _I, _PI, C.c_int, C.POINTER(_P), C.POINTER(_P)],
    "ttn_block_destroy": [_P],
    "ttn_block_node_size": [_P, _I, C.POINTER(C.c_int64)],
    "ttn_envs_create": [_P, _P, _I, _PI, _PI, _PI, C.c_int, C.POINTER(_P), C.POINTER(_P)],
    "ttn_envs_destroy": [_P],
    "ttno_env_update": [_P, _P, _P, _P, _P, _I, _P, _P, _I, _I, _P, C.c_int],
    "ttno_env_close": [_P, _P, _P, _P, _P, _I, _P, _P, _I, _P, _P, C.c_int],
    "heff_apply_block": [_P, _P, _P, _P, _I, _I, _P, _P, _P, _P, _P, _I, _P, C.c_uint32, C.c_int],
    "heff_apply_block_noalloc": [_P, _P, _P, _P, _I, _I, _P, _P, _P, _P, _P, _I, _P, C.c_uint32, C.c_int],
    "rayleigh_ritz": [_P, _I, _PI, _I, _P, _P, _I, C.c_double, _I, _P, _P, _P],
    "ttn_block_move_centre": [_P, _P, _I, _I],
    "ttn_block_scale_node": [_P, _P, _I, _P],
    "ttn_block_node_norms2": [_P, _P, _I, _P],
    "ttn_sop_build": [_P, _PI, _I, C.POINTER(C.c_double), _PI, _I, _PI, _PI, _PI, C.POINTER(C.c_double),
                      C.c_double, C.POINTER(_P)],
    "ttn_sop_build_sd": [_P, _PI, _I, C.POINTER(C.c_double), _PI, _I, _PI, _PI, _PI, C.POINTER(C.c_double),
                         C.POINTER(_P)],
    "ttn_sop_bonds": [_P, _PI],
    "ttn_sop_tensor": [_P, _I, C.POINTER(C.c_double), C.c_int64],
    "ttn_sop_destroy": [_P],
    "ttn_flops_heff": [_P, _P, _P, _P, _I, _I, C.POINTER(C.c_double)],
    "ttn_flops_env": [_P, _P, _P, _P, _P, _I, _I, C.POINTER(C.c_double)],
    "ttn_sweep_create": [_P, _P, _P, _P, _I, C.POINTER(_P), C.POINTER(_P), _PI, C.POINTER(_P), C.POINTER(_P),
                         C.POINTER(_P), _P, C.c_int, C.POINTER(_P)],
    "ttn_sweep_init": [_P, _I],
    "ttn_sweep_destroy": [_P],
    "sweep_step": [_P, _P, _I, _I, _P, _P, _P],
    "ttn_block_normalize_node": [_P, _P, _I, _P],
    "ttn_scatter_sym": [_P, _I, _P, _P, _P, _P],
    "ttn_vec_scale": [_P, _I, _P, C.c_double, _P],
    "ttn_ctx_profile": [_P, _I],
    "ttn_ctx_flops": [_P, C.POINTER(C.c_double), _I],
    "ttn_alloc_count": [C.POINTER(C.c_int64)],
    "ttn_src_bonds": [_P, _I, _P],
    "ttn_src_create": [_P, _P, _P, _P, _P, _I, C.c_int, _P],
    "ttn_src_apply": [_P, _P, _P],
    "ttn_src_destroy": [_P],
    "ttn_expand_create": [_P, _P, _P, _P, _P, _I, C.c_int, _P],
    "ttn_expand_apply": [_P, _P, _P],
    "ttn_expand_destroy": [_P],
    "ttn_ctx_profile_filter": [_P, _I, _P],
    "ttn_ctx_probe_heff": [_P, _I, _P],
    "ttn_ctx_probe_report": [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "ttn_vec_sqrt": [_P, _I, _P, _P],
    "ttn_vec_gather": [_P, _I, _P, _P, _I, C.c_double, _P],
    "ttn_block_convert": [_P, _P, _P, _I],
    "ttn_ctx_profile_report": [_P, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)],
    "ttn_mlp_forward": [_P, _P, _I, _P, _P, _P, C.c_int],
    "ttn_mlp_backward": [_P, _P, _I, _P, _P, _P, _P, C.c_int],
    "ttn_mlp_loss": [_P, _I, _P, _P, _P, _P],
    "ttn_mlp_adam": [_P, _P, _P, _P, _P, C.c_float, C.c_float, C.c_float, C.c_float, _I],
    "ttn_precond_features": [_P, _I, C.c_int64, C.c_int, _P, _P, _P, _P],
    "ttn_precond_targets": [_P, _I, C.c_int64, C.c_int, _P, _P, _P, _P, _P],
    "ttn_sweep_harvest": [_P, _P, _I, _P, _P, _P],
    "ttn_sweep_run": [_P, _P, _P, _I, _I, _I, _P, _P],
    "ttn_ctx_autotune": [_P, _I, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)],
}


def lib():
    """Load libttn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_15875_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int32
        L.ttn_last_error.argtypes = [_P]
        L.ttn_last_error.restype = C.c_char_p
        L.ttn_version.argtypes = []
        L.ttn_version.restype = C.c_char_p
        L.ttn_mlp_num_params.argtypes = []
        L.ttn_mlp_num_params.restype = C.c_int64
        _lib = L
    return _lib


# ttn_status codes (include/ttn.h)
OK, E_ARG, E_SHAPE, E_DTYPE, E_DEVICE, E_WORKSPACE, E_LAUNCH, E_NOT_PD, E_NONFINITE, E_NOCONV = range(10)


class TTNError(RuntimeError):
    def __init__(self, msg: str, status: int = -1):
        super().__init__(msg)
        self.status = status


def _check(status, ctx=None):
    if status != 0:
        msg = lib().ttn_last_error(ctx.h if ctx is not None else None)
        raise TTNError(f"ttn status {status}: {msg.decode() if msg else ''}", int(status))


def _i32(seq) -> C.Array:
    arr = (C.c_int32 * len(seq))(*[int(x) for x in seq])
    return arr


def _ptrs(seq) -> C.Array:
    return (C.c_void_p * len(seq))(*[(None if x is None else int(x)) for x in seq])


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def torch_dtype(dt: int):
    return torch.float64 if dt == F64 else torch.float32


class Context:
    def __init__(self, device: int = 0, workspace_bytes: int = 1 << 30, stream=None):
        self.h = C.c_void_p()
        s = stream if stream is not None else torch.cuda.current_stream(device)
        _check(lib().ttn_ctx_create(device, C.c_void_p(s.cuda_stream), workspace_bytes, C.byref(self.h)))
        self.device = device
        self._sweeps = weakref.WeakSet()

    def set_stream(self, stream):
        _check(lib().ttn_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)), self)

    def sync(self):
        _check(lib().ttn_ctx_sync(self.h), self)

    def close(self):
        """Destroy the context; sweeps created on it are destroyed first (a
        sweep keeps a pointer to its context)."""
        if self.h:
            for sw in list(self._sweeps):
                sw.close()
            lib().ttn_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    def __init__(self, parent: Sequence[int], phys: Sequence[int]):
        self.parent = list(parent)
        self.phys = list(phys)
        self.n = len(parent)
        self.h = C.c_void_p()
        _check(lib().ttn_tree_create(self.n, _i32(parent), _i32(phys), C.byref(self.h)))
        self.children = [[v for v in range(self.n) if self.parent[v] == u] for u in range(self.n)]
        self.root = self.parent.index(-1)

    def nbrs(self, u):
        return ([self.parent[u]] if self.parent[u] >= 0 else []) + self.children[u]

    def __del__(self):
        try:
            lib().ttn_tree_destroy(self.h)
        except Exception:
            pass


def dslot(tree: Tree, u: int, v: int) -> int:
    """Directed-edge slot of u -> v."""
    return 2 * u if tree.parent[u] == v else 2 * v + 1


class TTNO:
    """TTNO handle over caller-owned device tensors W[u] (legs [w_N..., p, q])."""

    def __init__(self, ctx: Context, tree: Tree, W: List[torch.Tensor], op_bond: Sequence[int], dtype: int):
        self.W = W
        self.M = list(op_bond)
        self.dtype = dtype
        self.h = C.c_void_p()
        _check(lib().ttn_ttno_create(ctx.h, tree.h, _i32(op_bond), dtype, _ptrs([w.data_ptr() for w in W]),
                                     C.byref(self.h)), ctx)

    def __del__(self):
        try:
            lib().ttn_ttno_destroy(self.h)
        except Exception:
            pass


class Block:
    """k states; node u stored as a [k, *legdims(u)] device tensor."""

    def __init__(self, ctx: Context, tree: Tree, k: int, bond: Sequence[int], dtype: int,
                 tensors: Optional[List[torch.Tensor]] = None, device="cuda"):
        self.tree, self.k, self.bond, self.dtype = tree, k, list(bond), dtype
        if tensors is None:
            tensors = [torch.zeros((k,) + tuple(self.legdims(u)), dtype=torch_dtype(dtype), device=device)
                       for u in range(tree.n)]
        self.t = tensors
        self.h = C.c_void_p()
        _check(lib().ttn_block_create(ctx.h, tree.h, k, _i32(bond), dtype, _ptrs([x.data_ptr() for x in tensors]),
                                      C.byref(self.h)), ctx)

    def legdims(self, u):
        tr = self.tree
        d = []
        for v in tr.nbrs(u):
            d.append(self.bond[u] if tr.parent[u] == v else self.bond[v])
        d.append(tr.phys[u])
        return d

    def __del__(self):
        try:
            lib().ttn_block_destroy(self.h)
        except Exception:
            pass


class Envs:
    """Environment slots: directed edge s holds [n_slots, Db, M, Da]."""

    def __init__(self, ctx: Context, tree: Tree, n_slots: int, bra_bond, op_bond, ket_bond, dtype: int,
                 edges: Optional[Sequence] = None, device="cuda"):
        self.tree, self.n_slots, self.dtype = tree, n_slots, dtype
        self.Db, self.Da = list(bra_bond), list(ket_bond)
        self.M = list(op_bond) if op_bond is not None else [1] * tree.n
        self.slots: List[Optional[torch.Tensor]] = [None] * (2 * tree.n)
        for u in range(tree.n):
            if tree.parent[u] < 0:
                continue
            for s in (2 * u, 2 * u + 1):
                if edges is not None and s not in edges:
                    continue
                self.slots[s] = torch.zeros((n_slots, self.Db[u], self.M[u], self.Da[u]),
                                            dtype=torch_dtype(dtype), device=device)
        self.h = C.c_void_p()
        _check(lib().ttn_envs_create(ctx.h, tree.h, n_slots, _i32(bra_bond),
                                     None if op_bond is None else _i32(op_bond), _i32(ket_bond), dtype,
                                     _ptrs([None if x is None else x.data_ptr() for x in self.slots]),
                                     C.byref(self.h)), ctx)

    def get(self, u, v) -> torch.Tensor:
        return self.slots[dslot(self.tree, u, v)]

    def __del__(self):
        try:
            lib().ttn_envs_destroy(self.h)
        except Exception:
            pass


# ---------------------------------------------------------------- hot-path calls

def ttno_env_update(ctx: Context, tree: Tree, op: Optional[TTNO], bra: Block, ket: Block, pair_bra: torch.Tensor,
                    pair_ket: torch.Tensor, node: int, toward: int, envs: Envs, compute: int):
    n = int(pair_bra.numel())
    _check(lib().ttno_env_update(ctx.h, tree.h, None if op is None else op.h, bra.h, ket.h, n, _ptr(pair_bra),
                                 _ptr(pair_ket), node, toward, envs.h, compute), ctx)


def ttno_env_close(ctx: Context, tree: Tree, op: Optional[TTNO], bra: Block, ket: Block, pair_bra: torch.Tensor,
                   pair_ket: torch.Tensor, node: int, envs: Envs, out: torch.Tensor, compute: int):
    n = int(pair_bra.numel())
    _check(lib().ttno_env_close(ctx.h, tree.h, None if op is None else op.h, bra.h, ket.h, n, _ptr(pair_bra),
                                _ptr(pair_ket), node, envs.h, _ptr(out), compute), ctx)


def heff_apply_block(ctx: Context, tree: Tree, op: Optional[TTNO], envs: Envs, node: int, k: int,
                     X: Optional[torch.Tensor], Y: torch.Tensor, pair_ids=None, x_ids=None, shift=None, alpha=None,
                     flags: int = HEFF_APPLY, compute: int = F64):
    x_rows = int(X.shape[0]) if X is not None else 0
    _check(lib().heff_apply_block(ctx.h, tree.h, None if op is None else op.h, envs.h, node, k, _ptr(pair_ids),
                                  _ptr(x_ids), _ptr(shift), _ptr(alpha), _ptr(X), x_rows, _ptr(Y), flags,
                                  compute), ctx)


def heff_apply_block_noalloc(ctx: Context, tree: Tree, op: Optional[TTNO], envs: Envs, node: int, k: int,
                             X: Optional[torch.Tensor], Y: torch.Tensor, pair_ids=None, x_ids=None, shift=None,
                             alpha=None, flags: int = HEFF_APPLY, compute: int = F64):
    """heff_apply_block with the library's static device scratch as workspace (allocates nothing)."""
    x_rows = int(X.shape[0]) if X is not None else 0
    _check(lib().heff_apply_block_noalloc(ctx.h, tree.h, None if op is None else op.h, envs.h, node, k,
                                          _ptr(pair_ids), _ptr(x_ids), _ptr(shift), _ptr(alpha), _ptr(X), x_rows,
                                          _ptr(Y), flags, compute), ctx)


def flops_heff(tree: Tree, op: Optional[TTNO], envs: Envs, node: int, k: int) -> float:
    out = C.c_double()
    _check(lib().ttn_flops_heff(None, tree.h, None if op is None else op.h, envs.h, node, k, C.byref(out)))
    return out.value


def flops_env(tree: Tree, op: Optional[TTNO], bra: Block, ket: Block, node: int, toward: int) -> float:
    out = C.c_double()
    _check(lib().ttn_flops_env(None, tree.h, None if op is None else op.h, bra.h, ket.h, node, toward,
                               C.byref(out)))
    return out.value


def rayleigh_ritz(ctx: Context, H: torch.Tensor, S: torch.Tensor, m: Sequence[int], nev: int,
                  drop_tol: float = 1e-12, allow_svqb: bool = True):
    """H, S: [batch, ld, ld] float64 device tensors.  Returns (evals, V, rank)."""
    batch, ld = H.shape[0], H.shape[1]
    evals = torch.empty((batch, nev), dtype=torch.float64, device=H.device)
    V = torch.empty((batch, ld, nev), dtype=torch.float64, device=H.device)
    rank = torch.empty((batch,), dtype=torch.int32, device=H.device)
    _check(lib().rayleigh_ritz(ctx.h, batch, _i32(m), ld, _ptr(H), _ptr(S), nev, drop_tol, 1 if allow_svqb else 0,
                               _ptr(evals), _ptr(V), _ptr(rank)), ctx)
    return evals, V, rank


def block_move_centre(ctx: Context, b: Block, u: int, v: int):
    _check(lib().ttn_block_move_centre(ctx.h, b.h, u, v), ctx)


def block_scale_node(ctx: Context, b: Block, u: int, scale: torch.Tensor):
    _check(lib().ttn_block_scale_node(ctx.h, b.h, u, _ptr(scale)), ctx)


def block_node_norms2(ctx: Context, b: Block, u: int, out: torch.Tensor):
    _check(lib().ttn_block_node_norms2(ctx.h, b.h, u, _ptr(out)), ctx)


def sop_build(tree: Tree, node_mode: Sequence[int], omega, dims, monomials, coefs, rel_tol: float = 1e-13,
              method: str = "svd"):
    """Compile a sum-of-products Hamiltonian to TTNO tensors on the host (FP64):
    method "svd" (channel automaton compressed to the operator Schmidt rank) or
    "state_diagram" (minimum vertex covers, uncompressed and sparse).
    Returns (list of numpy arrays W[u], op_bond list)."""
    import numpy as np
    n_modes = len(omega)
    ptr, mm, pw = [0], [], []
    for mono in monomials:
        for m, p in mono:
            mm.append(m)
            pw.append(p)
        ptr.append(len(mm))
    h = C.c_void_p()
    om = (C.c_double * n_modes)(*[float(x) for x in omega])
    cf = (C.c_double * max(1, len(coefs)))(*[float(x) for x in coefs])
    if method == "svd":
        _check(lib().ttn_sop_build(tree.h, _i32(node_mode), n_modes, om, _i32(dims), len(monomials), _i32(ptr),
                                   _i32(mm if mm else [0]), _i32(pw if pw else [0]), cf, rel_tol, C.byref(h)))
    elif method == "state_diagram":
        _check(lib().ttn_sop_build_sd(tree.h, _i32(node_mode), n_modes, om, _i32(dims), len(monomials), _i32(ptr),
                                      _i32(mm if mm else [0]), _i32(pw if pw else [0]), cf, C.byref(h)))
    else:
        raise ValueError("method: 'svd' or 'state_diagram'")
    try:
        bonds = (C.c_int32 * tree.n)()
        _check(lib().ttn_sop_bonds(h, bonds))
        bonds = list(bonds)
        W = []
        for u in range(tree.n):
            shp = []
            for v in tree.nbrs(u):
                shp.append(bonds[u] if tree.parent[u] == v else bonds[v])
            shp += [tree.phys[u], tree.phys[u]]
            buf = np.zeros(int(np.prod(shp)), dtype=np.float64)
            _check(lib().ttn_sop_tensor(h, u, buf.ctypes.data_as(C.POINTER(C.c_double)), buf.size))
            W.append(buf.reshape(shp))
        return W, bonds
    finally:
        lib().ttn_sop_destroy(h)


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("maxiter", C.c_int32), ("rtol", C.c_double), ("mlp_params", C.c_void_p),
                ("mlp_compute", C.c_int32), ("refine", C.c_int32), ("learned_coef", C.c_void_p), ("warm", C.c_int32),
                ("precond", C.c_int32), ("precond_damp", C.c_double)]


class Sweep:
    """A sweep of local solves over a target block (see ttn_sweep_create).

    sources: list of (op or None, Block, targets, sources, coef device tensor or None)."""

    def __init__(self, ctx: Context, tree: Tree, op: Optional[TTNO], target: Block, sources, shift=None,
                 compute: int = F64):
        self.ctx, self.tree, self.target = ctx, tree, target
        self._keep = [op, target, sources, shift]
        n = len(sources)
        ops = (C.c_void_p * max(1, n))(*[(s[0].h.value if s[0] is not None else None) for s in sources])
        blks = (C.c_void_p * max(1, n))(*[s[1].h.value for s in sources])
        nt = _i32([len(s[2]) for s in sources] or [0])
        tg = [_i32(s[2]) for s in sources]
        sr = [_i32(s[3]) for s in sources]
        self._arrs = (tg, sr)
        tgp = (C.c_void_p * max(1, n))(*[C.cast(a, C.c_void_p).value for a in tg])
        srp = (C.c_void_p * max(1, n))(*[C.cast(a, C.c_void_p).value for a in sr])
        cfp = (C.c_void_p * max(1, n))(*[(s[4].data_ptr() if s[4] is not None else None) for s in sources])
        self.h = C.c_void_p()
        _check(lib().ttn_sweep_create(ctx.h, tree.h, None if op is None else op.h, target.h, n, ops, blks, nt, tgp,
                                      srp, cfp, _ptr(shift), compute, C.byref(self.h)), ctx)
        ctx._sweeps.add(self)

    def init(self, centre: int):
        _check(lib().ttn_sweep_init(self.h, centre), self.ctx)

    def step(self, node: int, nxt: int, mode: int, maxiter: int = 0, rtol: float = 0.0, iters=None, resid=None,
             mlp: Optional[torch.Tensor] = None, mlp_compute: int = BF16, learned_coef=None, refine: int = 0,
             warm: int = 0, precond: int = 0, precond_damp: float = 0.0):
        o = SolveOpts(mode, maxiter, rtol, None if mlp is None else mlp.data_ptr(), mlp_compute, refine,
                      None if learned_coef is None else learned_coef.data_ptr(), warm, precond, precond_damp)
        _check(lib().sweep_step(self.ctx.h, self.h, node, nxt, C.byref(o), _ptr(iters), _ptr(resid)), self.ctx)

    def run(self, mode: int, n_sweeps: int = 1, init: bool = False, graph: bool = False, maxiter: int = 0,
            rtol: float = 0.0, iters=None, resid=None, mlp: Optional[torch.Tensor] = None, mlp_compute: int = BF16,
            refine: int = 0, warm: int = 0, precond: int = 0, precond_damp: float = 0.0):
        """n_sweeps native sweeps (see ttn_sweep_run), optionally replayed as a HIP graph."""
        o = SolveOpts(mode, maxiter, rtol, None if mlp is None else mlp.data_ptr(), mlp_compute, refine, None, warm,
                      precond, precond_damp)
        _check(lib().ttn_sweep_run(self.ctx.h, self.h, C.byref(o), n_sweeps, int(init), int(graph), _ptr(iters),
                                   _ptr(resid)), self.ctx)

    def harvest(self, node: int, X: torch.Tensor, T: torch.Tensor, scales: torch.Tensor):
        """Training pairs of the current local problems at `node` (see ttn_sweep_harvest)."""
        _check(lib().ttn_sweep_harvest(self.ctx.h, self.h, node, _ptr(X), _ptr(T), _ptr(scales)), self.ctx)

    def close(self):
        if self.h:
            lib().ttn_sweep_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def euler_tour(tree: Tree):
    out = []

    def rec(u):
        out.append(u)
        for c in tree.children[u]:
            rec(c)
            out.append(u)

    rec(tree.root)
    return out


def run_sweep(sw: Sweep, tree: Tree, mode: int, maxiter: int = 0, rtol: float = 0.0, iters=None, resid=None,
              collect=None, mlp=None, mlp_compute: int = BF16, on_solved=None, refine: int = 0, precond: int = 0,
              precond_damp: float = 0.0):
    """One sweep: a depth-first Euler tour from the root; a node is solved on
    its first visit, later visits only move the orthogonality centre.
    collect: optional list receiving (node, iters tensor) per local solve.
    on_solved(u): optional callback after a node's local solve, before the
    centre moves on (harvesting reads the local problem there)."""
    if collect is None and on_solved is None:
        sw.run(mode, 1, maxiter=maxiter, rtol=rtol, iters=iters, resid=resid, mlp=mlp, mlp_compute=mlp_compute,
               refine=refine, precond=precond, precond_damp=precond_damp)
        return
    tour = euler_tour(tree)
    seen = set()
    for t, u in enumerate(tour):
        nxt = tour[t + 1] if t + 1 < len(tour) else -1
        m = mode if u not in seen else SOLVE_SKIP
        if on_solved is not None and m != SOLVE_SKIP:
            sw.step(u, -1, m, maxiter, rtol, iters, resid, mlp, mlp_compute)
            on_solved(u)
            sw.step(u, nxt, SOLVE_SKIP)
        elif collect is not None and m == SOLVE_MINRES:
            it = torch.zeros(sw.target.k, dtype=torch.int32, device="cuda")
            sw.step(u, nxt, m, maxiter, rtol, it, resid, refine=refine, precond=precond, precond_damp=precond_damp)
            collect.append((u, it))
        else:
            sw.step(u, nxt, m, maxiter, rtol, iters, resid, mlp, mlp_compute)
        seen.add(u)


def ctx_flops(ctx: Context, reset: bool = False) -> float:
    out = C.c_double()
    _check(lib().ttn_ctx_flops(ctx.h, C.byref(out), 1 if reset else 0), ctx)
    return out.value


def profile(ctx: Context, on: bool):
    _check(lib().ttn_ctx_profile(ctx.h, 1 if on else 0), ctx)


def profile_filter(ctx: Context, prefixes: Sequence[str]):
    """Record only plans whose key starts with one of the prefixes (empty: all)."""
    arr = (C.c_char_p * max(1, len(prefixes)))(*[p.encode() for p in prefixes])
    _check(lib().ttn_ctx_profile_filter(ctx.h, len(prefixes), C.cast(arr, C.c_void_p)), ctx)


def probe_heff(ctx: Context, nodes: Sequence[int]):
    """Bracket every heff_apply_block call with the operator at these nodes by HIP events."""
    arr = _i32(list(nodes) or [0])
    _check(lib().ttn_ctx_probe_heff(ctx.h, len(nodes), C.cast(arr, C.c_void_p)), ctx)


def probe_report(ctx: Context):
    """(calls, algorithmic flops, summed event ms) of the probed heff_apply_block calls since the last report."""
    n, f, ms = C.c_int64(), C.c_double(), C.c_double()
    _check(lib().ttn_ctx_probe_report(ctx.h, C.byref(n), C.byref(f), C.byref(ms)), ctx)
    return int(n.value), float(f.value), float(ms.value)


def profile_report(ctx: Context):
    """[(plan_key, stage, kernel, launches, total_ms, flops, M, N, K, batch_items, bytes)] since the last
    report (bytes: compulsory bytes, see ttn_ctx_profile_report)."""
    need = C.c_int64()
    _check(lib().ttn_ctx_profile_report(ctx.h, None, 0, C.byref(need)), ctx)
    buf = C.create_string_buffer(int(need.value) + 1024)
    _check(lib().ttn_ctx_profile_report(ctx.h, buf, len(buf), C.byref(need)), ctx)
    out = []
    for line in buf.value.decode().splitlines():
        k, st, kern, cnt, ms, fl, M, N, K, nz, by = line.split("|")
        out.append((k, int(st), kern, int(cnt), float(ms), float(fl), int(M), int(N), int(K), int(nz), float(by)))
    return out


def block_normalize_node(ctx: Context, b: Block, u: int, norms=None):
    _check(lib().ttn_block_normalize_node(ctx.h, b.h, u, _ptr(norms)), ctx)


def scatter_sym(ctx: Context, idx_a: torch.Tensor, idx_b: torch.Tensor, vals: torch.Tensor, out: torch.Tensor):
    _check(lib().ttn_scatter_sym(ctx.h, int(idx_a.numel()), _ptr(idx_a), _ptr(idx_b), _ptr(vals), _ptr(out)), ctx)


def vec_sqrt(ctx: Context, x: torch.Tensor, y: torch.Tensor):
    _check(lib().ttn_vec_sqrt(ctx.h, int(x.numel()), _ptr(x), _ptr(y)), ctx)


def vec_gather(ctx: Context, idx: torch.Tensor, src: torch.Tensor, dst: torch.Tensor, fill: float = 0.0):
    """dst[i] = src[idx[i]] (idx[i] >= 0) else fill, on the device (ttn_vec_gather)."""
    _check(lib().ttn_vec_gather(ctx.h, int(idx.numel()), _ptr(idx), _ptr(src), int(src.numel()), float(fill),
                                _ptr(dst)), ctx)


def block_convert(ctx: Context, src: "Block", dst: "Block", rows: int):
    _check(lib().ttn_block_convert(ctx.h, src.h, dst.h, int(rows)), ctx)


def vec_scale(ctx: Context, x: torch.Tensor, alpha: float, y: torch.Tensor):
    _check(lib().ttn_vec_scale(ctx.h, int(x.numel()), _ptr(x), float(alpha), _ptr(y)), ctx)


def src_bonds(tree: Tree, chi: int) -> List[int]:
    """Bonds of the state successive randomized compression produces with sketch size chi."""
    out = (C.c_int32 * tree.n)()
    _check(lib().ttn_src_bonds(tree.h, int(chi), C.cast(out, C.c_void_p)))
    return list(out)


class Src:
    """Successive randomized compression y_j ~ H x_j of a block (ttn_src_*)."""

    def __init__(self, ctx: Context, tree: Tree, op: "TTNO", x: "Block", y: "Block", chi: int, compute: int):
        self.ctx, self.tree, self.chi = ctx, tree, chi
        self.h = C.c_void_p()
        _check(lib().ttn_src_create(ctx.h, tree.h, op.h, x.h, y.h, int(chi), int(compute), C.byref(self.h)), ctx)

    def apply(self, omegas: Sequence[Optional[torch.Tensor]]):
        """omegas[u]: device [chi][phys_u] test matrix rows of physical node u (None at auxiliary nodes)."""
        self._keep = list(omegas)
        arr = _ptrs([None if o is None else o.data_ptr() for o in omegas])
        _check(lib().ttn_src_apply(self.ctx.h, self.h, C.cast(arr, C.c_void_p)), self.ctx)

    def close(self):
        if self.h:
            lib().ttn_src_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Expand:
    """Bond expansion x -> y (larger bonds, same states) from the residual of
    the local H x (ttn_expand_*)."""

    def __init__(self, ctx: Context, tree: Tree, op: "TTNO", x: "Block", y: "Block", n_sketch: int, compute: int):
        self.ctx, self.tree, self.n = ctx, tree, n_sketch
        self.h = C.c_void_p()
        _check(lib().ttn_expand_create(ctx.h, tree.h, op.h, x.h, y.h, int(n_sketch), int(compute),
                                       C.byref(self.h)), ctx)

    def apply(self, omegas: Sequence[Optional[torch.Tensor]]):
        """omegas[u]: device [n_sketch][phys_u] sketch rows of physical node u (None at auxiliary nodes)."""
        self._keep = list(omegas)
        arr = _ptrs([None if o is None else o.data_ptr() for o in omegas])
        _check(lib().ttn_expand_apply(self.ctx.h, self.h, C.cast(arr, C.c_void_p)), self.ctx)

    def close(self):
        if self.h:
            lib().ttn_expand_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def alloc_count() -> int:
    """Device and pinned-host allocations the library has made in this process."""
    out = C.c_int64()
    _check(lib().ttn_alloc_count(C.byref(out)))
    return int(out.value)


def version() -> str:
    return lib().ttn_version().decode()


# ---------------------------------------------------------------- learned local preconditioner

MLP_IN, MLP_HID, MLP_OUT, MLP_TILE = 128, 256, 64, 64


def mlp_num_params() -> int:
    return int(lib().ttn_mlp_num_params())


def mlp_forward(ctx: Context, params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, acts=None, compute: int = BF16):
    _check(lib().ttn_mlp_forward(ctx.h, _ptr(params), X.shape[0], _ptr(X), _ptr(Y), _ptr(acts), compute), ctx)


def mlp_backward(ctx: Context, params: torch.Tensor, X: torch.Tensor, acts: torch.Tensor, dY: torch.Tensor,
                 grads: torch.Tensor, compute: int = BF16):
    _check(lib().ttn_mlp_backward(ctx.h, _ptr(params), X.shape[0], _ptr(X), _ptr(acts), _ptr(dY), _ptr(grads),
                                  compute), ctx)


def mlp_loss(ctx: Context, Y: torch.Tensor, T: torch.Tensor, dY: torch.Tensor, loss: torch.Tensor):
    _check(lib().ttn_mlp_loss(ctx.h, Y.shape[0], _ptr(Y), _ptr(T), _ptr(dY), _ptr(loss)), ctx)


def mlp_adam(ctx: Context, params, m, v, grads, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8):
    _check(lib().ttn_mlp_adam(ctx.h, _ptr(params), _ptr(m), _ptr(v), _ptr(grads), lr, beta1, beta2, eps, step), ctx)


def precond_features(ctx: Context, b: torch.Tensor, d: torch.Tensor, scales: torch.Tensor, X: torch.Tensor):
    k, n = b.shape
    st = F64 if b.dtype == torch.float64 else F32
    _check(lib().ttn_precond_features(ctx.h, k, n, st, _ptr(b), _ptr(d), _ptr(scales), _ptr(X)), ctx)


def precond_targets(ctx: Context, y: torch.Tensor, b: torch.Tensor, d: torch.Tensor, scales: torch.Tensor,
                    T: torch.Tensor):
    k, n = y.shape
    st = F64 if y.dtype == torch.float64 else F32
    _check(lib().ttn_precond_targets(ctx.h, k, n, st, _ptr(y), _ptr(b), _ptr(d), _ptr(scales), _ptr(T)), ctx)


def autotune(ctx: Context, on: Optional[bool] = True) -> str:
    """Switch the tile autotuner (None: leave it) and return its log so far."""
    need = C.c_int64()
    flag = -1 if on is None else int(bool(on))
    _check(lib().ttn_ctx_autotune(ctx.h, flag, None, 0, C.byref(need)), ctx)
    buf = C.create_string_buffer(int(need.value) + 16)
    _check(lib().ttn_ctx_autotune(ctx.h, -1, buf, len(buf), C.byref(need)), ctx)
    return buf.value.decode()
