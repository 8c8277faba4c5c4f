"""Parity of the HIP Stokes ADMM path (through the C ABI) with the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import acm_oracle as O
from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, host, require_gpu


def _solve(H, g, **kw):
    from paper_2312_15554_amd.api import acm_stokes_solve
    return acm_stokes_solve(dev(H), g, **kw)


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(16, 16), (24, 32), (8, 24, 16), (16, 16, 16), (24, 16, 48)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_fixed_penalty_iterates_match_oracle(shape, dtype):
    """Same fixed penalties, same number of iterations: u and the six
    residuals of the HIP path equal the oracle's (Steps 1-4, Section 3.1)."""
    require_gpu()
    print(f"iterate parity shape={shape} dtype={dtype}", flush=True)
    H = I.random_mask(shape, 17, 0.35)
    d = len(shape)
    g = (1.0, 0.4, -0.3)[:d]
    pen = dict(alpha=30.0, beta=50.0, b=20.0, adaptive=0)
    M = 40
    r = _solve(H, g, dtype=dtype, penalty=pen, eps=0.0, max_iter=M)
    o = O.stokes_admm(H, g, alpha=30.0, beta=50.0, b=20.0, adaptive=False, eps=0.0, max_iter=M)
    assert r["stats"]["iters"] == M
    u = host(r["u"])
    scale = np.abs(o["u"]).max()
    tol = 1e-11 if dtype == torch.float64 else 2e-5
    assert np.abs(u - o["u"]).max() < tol * scale
    q = host(r["q"])
    assert np.abs(q - o["q"]).max() < tol * 10 * np.abs(o["q"]).max()
    for k in range(3):
        assert abs(r["stats"]["r_p"][k] - o["r_p"][k]) <= tol * 100 * (o["r_p"][k] + 1e-30) + 1e-12
        assert abs(r["stats"]["r_d"][k] - o["r_d"][k]) <= tol * 100 * (o["r_d"][k] + 1e-30) + 1e-12


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_poiseuille_closed_form(dtype):
    require_gpu()
    N, w = 32, 6
    H = I.slab_cell((16, N, 16), w, axis=1)
    prof = O.poiseuille_profile(N, w)
    eps = 1e-10 if dtype == torch.float64 else 1e-8
    r = _solve(H, (1.0, 0.0, 0.0), dtype=dtype, eps=eps, max_iter=200000)
    assert r["stats"]["converged"]
    u = host(r["u"])
    tol = 1e-7 if dtype == torch.float64 else 2e-5
    assert np.abs(u[0] - prof[None, :, None]).max() < tol * prof.max()
    assert np.abs(u[1:]).max() < tol * prof.max()


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_converged_permeability_matches_oracle(dtype):
    """Converged K tensor of a 16^3 overlapping-sphere cell vs the oracle at a
    tight tolerance (both reach the same discrete fixed point)."""
    require_gpu()
    H = I.overlapping_spheres(16, 1.0, 0.45, seed=3)
    eps = 1e-10 if dtype == torch.float64 else 1e-8
    us_gpu, us_or = [], []
    for g in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        r = _solve(H, g, dtype=dtype, eps=eps, max_iter=200000)
        assert r["stats"]["converged"], r["stats"]
        us_gpu.append(host(r["u"]).astype(np.float64))
        us_or.append(O.stokes_admm(H, g, eps=1e-11)["u"])
    Kg = O.permeability_darcy(us_gpu)
    Ko = O.permeability_darcy(us_or)
    rel = np.abs(Kg - Ko).max() / np.abs(Ko).max()
    assert rel < (1e-8 if dtype == torch.float64 else 1e-5), rel


@pytest.mark.gpu
def test_abi_error_codes():
    require_gpu()
    from paper_2312_15554_amd import abi
    from paper_2312_15554_amd.api import acm_stokes_solve
    Hf = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(abi.AcmError) as e:
        acm_stokes_solve(Hf, (1.0, 0.0))
    assert e.value.status == abi.ACM_E_INVALID
    Hb = torch.ones((20, 20), dtype=torch.uint8, device="cuda")
    with pytest.raises(abi.AcmError) as e:
        acm_stokes_solve(Hb, (1.0, 0.0))
    assert e.value.status == abi.ACM_E_UNSUPPORTED_SIZE
    H = dev(I.centred_disc(16))
    r = acm_stokes_solve(H, (1.0, 0.0), max_iter=1)
    assert r["status"] == abi.ACM_NOT_CONVERGED and r["stats"]["iters"] == 1
    assert torch.isfinite(r["u"]).all()
