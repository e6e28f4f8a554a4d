"""Many independent eigenproblems on one GPU.

Each member (its own Hamiltonian, tree, bond dimension and block size) gets
its own library context on its own HIP stream; a pool of host threads drives
the members' block-LOBPCG iterations concurrently (the library's calls
release the interpreter lock), so the members' uneven, mostly small launches
overlap on the device.  The sweeps of every iteration are replayed as HIP
graphs after their first runs, and the contraction tiles are picked by the
library's autotuner.  Phase two of the mixed form promotes each member to
FP64 for the refinement iterations.

The one-at-a-time baseline runs the same members, in order, on one stream
without graphs or tuning.
"""
from __future__ import annotations

import concurrent.futures as cf
import dataclasses
import time
from typing import List, Optional

import numpy as np
import torch

from . import ttn
from .solver import LobpcgOpts, MixedEigensolver, TTNEigensolver, build_ttno


@dataclasses.dataclass
class EnsembleOpts:
    low: str = "fp32"          # precision of the first phase ("fp32", "bf16" or "fp64" for plain)
    iters_low: int = 3         # LOBPCG iterations in the first phase
    iters_fp64: int = 1        # FP64 refinement iterations after promotion (0: none)
    concurrent: bool = True    # own stream per member + host thread pool
    threads: int = 8
    graphs: bool = True
    autotune: bool = True
    workspace_bytes: int = 1 << 30
    env_budget_bytes: int = 512 << 20  # Gram environments per solver


class Ensemble:
    def __init__(self, members: List[dict], opts: EnsembleOpts, log=None):
        import workloads as wl
        self.opts = opts
        self.members = members
        self.log = log
        self.items = []
        shared = None if opts.concurrent else torch.cuda.Stream()
        for m in members:
            st = torch.cuda.Stream() if opts.concurrent else shared
            with torch.cuda.stream(st):
                ctx = ttn.Context(0, workspace_bytes=opts.workspace_bytes, stream=st)
                ttn.autotune(ctx, opts.autotune)
                model = m["model"]
                tree = wl.binary_tree(model.dims) if m["kind"] == "c4-binary" else wl.fork_tree(model.dims, 4, 1)
                bonds = wl.bond_dims(tree, m["D"])
                x0 = wl.initial_block(tree, bonds, model.omega, model.dims, m["k"], m["seed"] + 17)
                if "ttno" not in m:
                    m["ttno"] = build_ttno(ttn.Tree(tree.parent, tree.phys), tree, model)
                if opts.iters_fp64 > 0 and opts.low != "fp64":
                    solver = MixedEigensolver(ctx, tree, model, D=m["D"], k=m["k"], low=opts.low, ttno=m["ttno"],
                                              env_budget_bytes=opts.env_budget_bytes)
                    solver.lo.graphs = solver.hi.graphs = opts.graphs
                else:
                    solver = TTNEigensolver(ctx, tree, model, D=m["D"], k=m["k"], precision=opts.low,
                                            graphs=opts.graphs, ttno=m["ttno"],
                                            env_budget_bytes=opts.env_budget_bytes)
                solver.load_block(x0)
            self.items.append({"stream": st, "ctx": ctx, "solver": solver, "tree": tree})
            if log:
                log(f"member {m['seed']} ({m['kind']}, L={m['L']}, D={m['D']}, k={m['k']}) ready")
        torch.cuda.synchronize()

    def _run_one(self, i: int):
        r = self._run(i)
        if self.log:
            self.log(f"member {self.members[i]['seed']} done")
        return r

    def _run(self, i: int):
        it = self.items[i]
        o = self.opts
        with torch.cuda.stream(it["stream"]):
            s = it["solver"]
            lo = s.lo if isinstance(s, MixedEigensolver) else s
            lo.lobpcg_start(LobpcgOpts(n_iter=o.iters_low + o.iters_fp64))
            for _ in range(o.iters_low):
                lo.lobpcg_step()
            if isinstance(s, MixedEigensolver):
                s.promote()
                for _ in range(o.iters_fp64):
                    s.hi.lobpcg_step()
                lam = s.hi.lam_d.cpu().numpy() + s.hi.zpe
            else:
                lam = lo.lam_d.cpu().numpy() + lo.zpe
            it["ctx"].sync()
        return np.sort(lam)

    def run(self):
        """All members' iterations; returns (eigenvalues per member, seconds, algorithmic flops)."""
        for it in self.items:
            ttn.ctx_flops(it["ctx"], reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if self.opts.concurrent:
            with cf.ThreadPoolExecutor(max_workers=self.opts.threads) as ex:
                lams = list(ex.map(self._run_one, range(len(self.items))))
        else:
            lams = [self._run_one(i) for i in range(len(self.items))]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        flops = sum(ttn.ctx_flops(it["ctx"]) for it in self.items)
        return lams, dt, flops

    def close(self):
        for it in self.items:
            it["ctx"].sync()
        self.items = []
