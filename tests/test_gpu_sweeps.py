"""The parameter-sweep harness (the shape of Section 4.1, Fig. pen_par, and
Section 4.2, Fig. comp_med) on small synthetic cells: what the method fixes
whatever the parameters."""
import numpy as np
import pytest
import torch

from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, require_gpu


@pytest.mark.gpu
@pytest.mark.parametrize("which", ["alpha", "beta", "b"])
def test_fixed_penalties_change_the_speed_not_the_fixed_point(which):
    """Model geometry (disc of radius 0.2) at 32^2, FP64, eps = 1e-11: every
    fixed setting of one penalty (0.5, 1, 2 times nu/h) and the adaptive
    schedule converge to the same permeability (Section 3.1: the ADMM fixed
    point is the constrained Stokes solution for any penalties), in different
    numbers of iterations."""
    require_gpu()
    from paper_2312_15554_amd.sweeps import penalty_sweep
    H = dev(I.centred_disc(32, 0.2))
    r = penalty_sweep(H, (1.0, 0.0), factors=(0.5, 1.0, 2.0), which=which, eps=1e-11,
                      max_iter=400000, tau=(20.0, 10.0, 30.0), dtype=torch.float64)
    print(f"  {which}: {r['fixed']} adaptive {r['adaptive']}", flush=True)
    assert all(it is not None for it in r["fixed"])
    ks = r["k_fixed"] + [r["k_adaptive"]]
    assert max(ks) - min(ks) < 1e-7 * abs(ks[0])
    assert "adaptive_psi_trace" in r and len(r["adaptive_psi_trace"]) > 0


@pytest.mark.gpu
def test_comparison_medium_sweep_shape():
    """Steady transport on the model geometry's flow (Pe = 10, eta = 0.01):
    above the smallest A0 for which the LS iteration converges, a larger A0
    converges more slowly (Section 4.2); in the flux form every convergent A0
    reaches the same solution, so its iterations measure speed only."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_stokes_solve
    from paper_2312_15554_amd.sweeps import comparison_medium_sweep
    H = dev(I.centred_disc(64, 0.2))
    r = acm_stokes_solve(H, (1.0, 0.0), eps=1e-7, max_iter=400000, want_q=False)
    u = r["u"]
    pore = (H == 0)
    ubar = torch.stack([(u[c] * pore).sum() / pore.sum() for c in range(2)]).double()
    un = (u / ubar.norm().float()).contiguous()
    for form in ("central", "flux"):
        res = comparison_medium_sweep(H, un, (1.0, 0.0), 10.0, A0s=(0.55, 1.1, 2.2, 4.4, 8.8),
                                      eps=1e-6, max_iter=20000, form=form)
        print(f"  {form}: {res['rows']}", flush=True)
        for row in res["rows"]:
            its = row["iters"]
            conv = [i for i, v in enumerate(its) if v is not None]
            assert conv, row
            best = min(conv, key=lambda i: its[i])
            assert its[-1] is not None and its[-1] > its[best]
