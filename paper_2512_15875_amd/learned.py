"""Training of the learned local preconditioner on the GPU.

The network (3 layers, 128 -> 256 -> 256 -> 64, SiLU) and its loss, gradient
and Adam update all run in the library's kernels (ttn_mlp_forward / _loss /
_backward / _adam); this module only keeps the device buffers, draws the
minibatch order and the initial weights (seeded inputs), and loops.
Parameters are FP32 master weights; the matrix-core arithmetic is BF16 by
default (operands rounded to bfloat16 as they are staged, FP32 accumulation).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from . import ttn

SIZES = [(128, 256), (256, 256), (256, 64)]


def init_params(seed: int) -> torch.Tensor:
    """Seeded He-normal weights (output layer scaled by 0.1), zero biases, as a
    device FP32 vector in the packed layout W1, b1, W2, b2, W3, b3."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    parts = []
    for li, (i, o) in enumerate(SIZES):
        scale = float(np.sqrt(2.0 / i)) * (0.1 if li == len(SIZES) - 1 else 1.0)
        parts += [torch.randn(i * o, generator=g, dtype=torch.float64) * scale, torch.zeros(o, dtype=torch.float64)]
    p = torch.cat(parts).to(device="cuda", dtype=torch.float32)
    assert p.numel() == ttn.mlp_num_params()
    return p


@dataclasses.dataclass
class TrainOpts:
    epochs: int = 20
    batch: int = 4096
    lr: float = 1e-3
    lr_final: float = 1e-4      # cosine decay from lr to lr_final
    val_frac: float = 0.1
    seed: int = 0
    compute: int = ttn.BF16


class Trainer:
    def __init__(self, ctx: ttn.Context, params: Optional[torch.Tensor] = None, seed: int = 0,
                 compute: int = ttn.BF16, max_batch: int = 8192):
        self.ctx = ctx
        self.compute = compute
        self.p = init_params(seed) if params is None else params.clone()
        P = self.p.numel()
        dev = "cuda"
        self.m = torch.zeros(P, dtype=torch.float32, device=dev)
        self.v = torch.zeros(P, dtype=torch.float32, device=dev)
        self.g = torch.zeros(P, dtype=torch.float32, device=dev)
        self.max_batch = max_batch
        self.acts = torch.empty(4, max_batch, 256, dtype=torch.float32, device=dev)
        self.Y = torch.empty(max_batch, 64, dtype=torch.float32, device=dev)
        self.dY = torch.empty(max_batch, 64, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.t = 0

    def step(self, X: torch.Tensor, T: torch.Tensor, lr: float) -> torch.Tensor:
        """One Adam step on a minibatch; returns the (device) loss before it."""
        n = X.shape[0]
        assert n <= self.max_batch and X.is_contiguous() and T.is_contiguous()
        acts = self.acts.view(-1)[: 4 * n * 256].view(4, n, 256)  # [4][n][256] contiguous
        Y, dY = self.Y[:n], self.dY[:n]
        ttn.mlp_forward(self.ctx, self.p, X, Y, acts, self.compute)
        ttn.mlp_loss(self.ctx, Y, T, dY, self.loss)
        ttn.mlp_backward(self.ctx, self.p, X, acts, dY, self.g, self.compute)
        self.t += 1
        ttn.mlp_adam(self.ctx, self.p, self.m, self.v, self.g, lr, self.t)
        return self.loss

    def evaluate(self, X: torch.Tensor, T: torch.Tensor) -> float:
        """Mean squared error over a data set (forward + loss kernels)."""
        tot, cnt = 0.0, 0
        for a in range(0, X.shape[0], self.max_batch):
            Xb, Tb = X[a:a + self.max_batch].contiguous(), T[a:a + self.max_batch].contiguous()
            n = Xb.shape[0]
            ttn.mlp_forward(self.ctx, self.p, Xb, self.Y[:n], None, self.compute)
            ttn.mlp_loss(self.ctx, self.Y[:n], Tb, self.dY[:n], self.loss)
            self.ctx.sync()
            tot += self.loss.item() * n
            cnt += n
        return tot / max(cnt, 1)

    def fit(self, X: torch.Tensor, T: torch.Tensor, opts: TrainOpts, log=None) -> List[dict]:
        """Adam over shuffled minibatches with a cosine learning-rate decay;
        a val_frac share of the pairs is held out.  Each epoch's record holds
        the training and validation MSE and, for scale, the MSE of the
        diagonal preconditioner's own prediction on the validation pairs."""
        n = X.shape[0]
        g = torch.Generator(device="cpu")
        g.manual_seed(opts.seed)
        perm = torch.randperm(n, generator=g).to(X.device)
        nv = int(round(opts.val_frac * n))
        Xv, Tv = X[perm[:nv]].contiguous(), T[perm[:nv]].contiguous()
        Xt, Tt = X[perm[nv:]].contiguous(), T[perm[nv:]].contiguous()
        nt = Xt.shape[0]
        steps_per_epoch = max(1, -(-nt // opts.batch))
        total = steps_per_epoch * opts.epochs
        hist = []
        k = 0
        for ep in range(opts.epochs):
            order = torch.randperm(nt, generator=g).to(X.device)
            for a in range(0, nt, opts.batch):
                idx = order[a:a + opts.batch]
                lr = opts.lr_final + 0.5 * (opts.lr - opts.lr_final) * (1 + np.cos(np.pi * k / total))
                self.step(Xt[idx].contiguous(), Tt[idx].contiguous(), float(lr))
                k += 1
            rec = {"epoch": ep, "train_mse": self.evaluate(Xt[:65536], Tt[:65536]),
                   "val_mse": self.evaluate(Xv, Tv) if nv else None,
                   "val_mse_diag": diag_mse(Xv, Tv) if nv else None}
            hist.append(rec)
            if log:
                log(rec)
        return hist


def diag_mse(X: torch.Tensor, T: torch.Tensor) -> float:
    """MSE of the diagonal preconditioner alone in network units: the targets
    are corrections over the DIAG step, so DIAG predicts zero."""
    return float((T.double() ** 2).mean().item())
