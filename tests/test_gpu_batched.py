"""Batched multi-cell Stokes solves (acm_stokes_solve_batched)."""
import numpy as np
import pytest
import torch

from oracle import acm_oracle as O
from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, host, require_gpu

CELLS = [((32, 32, 32), 1001), ((48, 48, 48), 1002), ((32, 32, 32), 1003), ((16, 16, 16), 1004),
         ((64, 64, 64), 1005)]


def _cells():
    out = []
    for shape, seed in CELLS:
        por = 0.3 + 0.3 * I.SplitMix64(seed).uniform()
        out.append(I.overlapping_spheres(shape, shape[-1] / 16.0, por, seed=seed))
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("pass_mode", [0, 1])
def test_batched_equals_single_cell_solves(pass_mode):
    """Each cell of a batch gets bit-for-bit the result of its own solve."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_stokes_solve, acm_stokes_solve_batched
    Hs = [dev(H) for H in _cells()]
    gs = [(1.0, 0.0, 0.0)] * len(Hs)
    # one green kernel for both calls: the autotuner's trial iterations (in
    # the first solve of a grid) run the other kernels, equal only to rounding
    rb = acm_stokes_solve_batched(Hs, gs, eps=1e-5, max_iter=20000, pass_mode=pass_mode,
                                  green_variant=1)
    for i, H in enumerate(Hs):
        print(f"batched cell {i} shape={tuple(H.shape)}", flush=True)
        # the pass structure the batch gave this cell: the fused slabs for
        # cubes that fit, else the separate x and y passes (a single cell of
        # another size would get the row-step passes)
        slab = H.shape[0] == H.shape[1] == H.shape[2] and H.shape[0] in (32, 48, 64, 96, 128)
        mode = pass_mode if (pass_mode != 0 or slab) else 1
        rs = acm_stokes_solve(H, gs[i], eps=1e-5, max_iter=20000, want_q=False, pass_mode=mode,
                              green_variant=1)
        assert rb["stats"][i]["converged"] and rs["stats"]["converged"]
        assert rb["stats"][i]["iters"] == rs["stats"]["iters"]
        assert torch.equal(rb["us"][i], rs["u"])


@pytest.mark.gpu
def test_batched_fixed_penalty_iterates_match_oracle():
    require_gpu()
    from paper_2312_15554_amd.api import acm_stokes_solve_batched
    Hn = [I.random_mask(s, k, 0.3) for s, k in [((16, 16, 16), 1), ((8, 24, 32), 2), ((16, 16, 16), 3)]]
    gs = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.2), (0.3, 0.3, 1.0)]
    qs = [torch.empty(H.shape, dtype=torch.float64, device="cuda") for H in Hn]
    M = 30
    rb = acm_stokes_solve_batched([dev(H) for H in Hn], gs, dtype=torch.float64,
                                  penalty=dict(alpha=30.0, beta=50.0, b=20.0, adaptive=0), eps=0.0,
                                  max_iter=M, qs=qs)
    for i, H in enumerate(Hn):
        o = O.stokes_admm(H, gs[i], alpha=30.0, beta=50.0, b=20.0, adaptive=False, eps=0.0, max_iter=M)
        assert rb["stats"][i]["iters"] == M
        assert np.abs(host(rb["us"][i]) - o["u"]).max() < 1e-11 * np.abs(o["u"]).max()
        assert np.abs(host(qs[i]) - o["q"]).max() < 1e-10 * np.abs(o["q"]).max()
