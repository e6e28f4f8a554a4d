"""heff_apply_block_noalloc (static device scratch, no allocation) against
heff_apply_block on the same inputs: two calls in a row, the second with a
smaller input, in FP32 and FP64; both against the oracle's K2 as well."""
import numpy as np
import pytest
import torch

from oracle import ttn as ottn
from tests.gpu_util import TOL, heff_setup, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2512_15875_amd import ttn
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ttn.lib()
    return ttn


# a level-2 node of the 64-mode binary tree, then a smaller MPS site
CALLS = [(3, 1, [24, 24, 24], [21, 14, 14], [24, 24, 24], 40), (2, 6, [8, 8], [5, 4], [8, 8], 5)]


@pytest.mark.parametrize("dt", [0, 1])
def test_noalloc_matches_heff_apply_block(api, dt):
    ctx = api.Context(0, workspace_bytes=1 << 30)
    for ci, (kappa, d, Db, M, Da, k) in enumerate(CALLS):
        tree, W, X, E, gt, gW, envs, tdt = heff_setup(api, ctx, kappa, d, Db, M, Da, k, 500 + ci, dt)
        shift = np.linspace(-1.0, 2.0, k)
        gX = to_dev(X, tdt)
        Y_ref = torch.zeros((k,) + tuple(Db) + (d,), dtype=tdt, device="cuda")
        Y_na = torch.full_like(Y_ref, float("nan"))
        api.heff_apply_block(ctx, gt, gW, envs, 1, k, gX, Y_ref, shift=to_dev(shift), compute=dt)
        ctx.sync()
        n_alloc = api.alloc_count()
        api.heff_apply_block_noalloc(ctx, gt, gW, envs, 1, k, gX, Y_na, shift=to_dev(shift), compute=dt)
        ctx.sync()
        assert api.alloc_count() == n_alloc
        # the same kernels on the same plan: identical per state
        assert torch.equal(Y_na, Y_ref), (ci, dt)
        for j in (0, k - 1):
            ein = {c: E[c][j] for c in tree.neighbours(1)}
            ref = ottn.heff_apply(tree, 1, W, X[j], ein, shift[j])
            assert rel_err(Y_na[j].double().cpu().numpy(), ref) < TOL[dt], (ci, dt, j)
    ctx.close()


def test_noalloc_rejects_oversized_state(api):
    """One state whose intermediates exceed the 256 MiB static array is
    refused with TTN_E_WORKSPACE before any launch (host-side check): at a
    two-leg node with bonds 512, operator bonds 64 and d = 8 every pairwise
    order has a first intermediate of 512 * 512 * 8 * 64 floats (537 MB)."""
    ctx = api.Context(0, workspace_bytes=1 << 30)
    kappa, d, Db, M, Da, k = 2, 8, [512, 512], [64, 64], [512, 512], 1
    tree, W, X, E, gt, gW, envs, tdt = heff_setup(api, ctx, kappa, d, Db, M, Da, k, 9, 1)
    Y = torch.zeros((k,) + tuple(Db) + (d,), dtype=tdt, device="cuda")
    with pytest.raises(api.TTNError) as ei:
        api.heff_apply_block_noalloc(ctx, gt, gW, envs, 1, k, to_dev(X, tdt), Y, compute=1)
    assert ei.value.status == api.E_WORKSPACE
    ctx.close()
