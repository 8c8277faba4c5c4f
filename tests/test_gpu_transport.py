"""Parity of the HIP Lippmann-Schwinger transport path and the effective
properties (through the C ABI) with the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import acm_oracle as O
from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, host, require_gpu


_FLOWS = {}


def _flow(H, g):
    key = (H.tobytes(), H.shape, tuple(g))
    if key not in _FLOWS:
        u, _ = O.brute_force_stokes(H, g)
        _FLOWS[key] = u / np.abs(u).max()
    return _FLOWS[key]


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(16, 16), (16, 24, 32), (16, 16, 16), (16, 32, 32), (8, 48, 48),
                                   (16, 64, 64), (8, 96, 96), (16, 128, 128), (8, 16, 256),
                                   (256, 8, 8)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dt", [math.inf, 5e-3])
def test_ls_iterates_match_oracle(shape, dtype, dt):
    """Fixed iteration count (eps = 0): chi of the HIP path equals the
    oracle's after the same LS iterations (eq. iter / eq. fft_solute).  Cubes
    in x-y with nx = ny in {32, 48, 64, 96, 128} take the slab form of the
    local pass (128 is the width of the timed cell), the others the row form
    with separate y passes."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_transport_step
    print(f"LS parity shape={shape} dtype={dtype} dt={dt}", flush=True)
    d = len(shape)
    H = I.random_mask(shape, 23, 0.3)
    u = I.random_field((d,) + shape, 29) * (1 - H)  # any advecting field will do here
    g = (0.3, 1.0, -0.5)[:d]
    B0 = (0.6, 0.0, 0.1)[:d]
    M, steps = 12, (1 if math.isinf(dt) else 3)
    r = acm_transport_step(dev(H), dev(u, dtype), g, 4.0, A0=0.55, B0=B0, eta=0.01, dt=dt,
                           n_steps=steps, eps=0.0, max_iter=M)
    o = O.transport_ls(H, u, g, 4.0, A0=0.55, B0=B0, eta=0.01, dt=dt, n_steps=steps, eps=0.0,
                       max_iter=M)
    assert r["stats"]["iters"] == M * steps
    chi = host(r["chi"])
    tol = 1e-11 if dtype == torch.float64 else 3e-5
    assert np.abs(chi - o["chi"]).max() < tol * np.abs(o["chi"]).max()


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_steady_transport_matches_brute_force(dtype):
    require_gpu()
    from paper_2312_15554_amd.api import acm_transport_step
    H = I.random_mask((16, 16, 16), 5, 0.3)
    u = _flow(H, (1.0, 0.0, 0.0))
    g = (1.0, 0.0, 0.0)
    ref = O.brute_force_transport(H, u, g, 5.0, A0=0.55, eta=0.01)
    eps = 1e-11 if dtype == torch.float64 else 1e-7
    r = acm_transport_step(dev(H), dev(u, dtype), g, 5.0, A0=0.55, B0=(1.0, 0, 0), eta=0.01,
                           eps=eps, max_iter=20000)
    assert r["stats"]["converged"]
    tol = 1e-7 if dtype == torch.float64 else 5e-5
    assert np.abs(host(r["chi"]) - ref).max() < tol * np.abs(ref).max()


@pytest.mark.gpu
def test_diffusion_mode_decay_closed_form():
    require_gpu()
    from paper_2312_15554_amd.api import acm_transport_step
    shape = (32, 32, 32)
    H = np.zeros(shape, np.uint8)
    u = np.zeros((3,) + shape)
    z, y, x = np.meshgrid(*[(np.arange(32) + 0.5) / 32] * 3, indexing="ij")
    mode = (1, 2, 1)
    chi0 = np.cos(2 * np.pi * (mode[0] * x + mode[1] * y + mode[2] * z))
    dt, n = 2e-3, 10
    r = acm_transport_step(dev(H), dev(u, torch.float32), (0.0, 0.0, 0.0), 0.0, A0=0.55, B0=(0, 0, 0),
                           dt=dt, n_steps=n, eps=1e-7, max_iter=500, chi=dev(chi0, torch.float32))
    amp = O.diffusion_mode_amplitude(shape, mode, dt, n, 0.55)
    assert r["stats"]["converged"]
    assert np.abs(host(r["chi"]) - amp * chi0).max() < 5e-6


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_effective_props_match_oracle_on_same_fields(dtype):
    require_gpu()
    from paper_2312_15554_amd.api import acm_effective_props
    shape = (16, 24, 32)
    H = I.random_mask(shape, 31, 0.35)
    us = [I.random_field((3,) + shape, s) * (1 - H) for s in (1, 2, 3)]
    chis = [I.random_field(shape, s) for s in (4, 5, 6)]
    r = acm_effective_props(dev(H), [dev(x, dtype) for x in us], [dev(x, dtype) for x in chis],
                            u_transport=dev(us[0], dtype), nu=0.7, Pe=3.0)
    cast = (lambda a: a.astype(np.float32).astype(np.float64)) if dtype == torch.float32 else (lambda a: a)
    Ko = O.permeability_darcy([cast(x) for x in us], nu=0.7)
    Do = O.effective_diffusivity(H, cast(us[0]), [cast(c) for c in chis], 3.0)
    mo = np.array([O.solute_mass(cast(c)) for c in chis])
    assert np.allclose(r["K"], Ko, rtol=1e-12, atol=1e-14)
    assert np.allclose(r["D"], Do, rtol=1e-12, atol=1e-13)
    assert np.allclose(r["mass"], mo, rtol=1e-12, atol=1e-14)


@pytest.mark.gpu
def test_mismatched_buffers_are_rejected_before_launch():
    require_gpu()
    from paper_2312_15554_amd.api import acm_stokes_solve, acm_transport_step
    H = dev(np.zeros((16, 16, 16), np.uint8))
    u64 = torch.zeros((3, 16, 16, 16), dtype=torch.float64, device="cuda")
    chi32 = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        acm_transport_step(H, u64, (1, 0, 0), 1.0, chi=chi32, max_iter=10)
    with pytest.raises(ValueError):
        acm_stokes_solve(H, (1, 0, 0), u=u64, max_iter=10)  # default dtype is float32
    with pytest.raises(ValueError):
        acm_transport_step(H, u64[:2].contiguous(), (1, 0, 0), 1.0, max_iter=10)


@pytest.mark.gpu
def test_exact_symbols_ring_where_central_symbols_do_not():
    """The paper's comparison of exact and approximate FFT derivatives
    (Section 4, Fig. model_sol d,e; the approximation of eq. fft_app):
    on the model geometry (circle of radius 0.2, 128^2, steady diffusion cell
    problem, eta = 0.01) the exact symbols leave spurious oscillations in the
    pore gradient field that the central symbols filter away.  Measured as
    the deviation of e_x + grad chi from the mean of its four neighbours, over
    pore voxels two or more voxels from the solid."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_transport_step
    print("exact vs central symbols: ringing on the model geometry", flush=True)
    n = 128
    y, x = np.meshgrid((np.arange(n) + 0.5) / n, (np.arange(n) + 0.5) / n, indexing="ij")
    H = (((x - 0.5) ** 2 + (y - 0.5) ** 2) < 0.2 ** 2).astype(np.uint8)
    u = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    pore = H == 0
    inner = pore.copy()
    for _ in range(2):
        inner = inner & np.roll(inner, 1, 0) & np.roll(inner, -1, 0) & np.roll(inner, 1, 1) & np.roll(inner, -1, 1)
    ring = {}
    for kind in ("central", "spectral"):
        r = acm_transport_step(dev(H), u, (1.0, 0.0), 0.0, A0=0.55, B0=(0.0, 0.0), eta=0.01,
                               eps=1e-9, max_iter=20000, derivative=kind)
        assert r["stats"]["converged"]
        chi = host(r["chi"])
        if kind == "central":
            dx = (np.roll(chi, -1, axis=1) - np.roll(chi, 1, axis=1)) * n / 2
        else:
            k = 2 * np.pi * np.fft.fftfreq(n, 1.0 / n)
            k[n // 2] = 0.0
            dx = np.real(np.fft.ifft(1j * k[None, :] * np.fft.fft(chi, axis=1), axis=1))
        gf = dx + 1.0
        nb = (np.roll(gf, 1, 0) + np.roll(gf, -1, 0) + np.roll(gf, 1, 1) + np.roll(gf, -1, 1)) / 4
        ring[kind] = float(np.abs(gf - nb)[inner].mean())
    print(f"  mean ringing: {ring}", flush=True)
    assert ring["spectral"] > 5.0 * ring["central"]


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(32, 32, 32), (16, 24, 32)])
def test_ls_divergence_is_reported(shape):
    """A comparison medium far below the largest diffusivity (A0 = 0.2 against
    A = 1 in the pore): the LS iteration grows, and the solve stops with
    ACM_E_DIVERGED once r_1 has grown a millionfold (Section 3.2: the
    iteration contracts only for a large enough A0).  The oracle diverges on
    the same cell."""
    require_gpu()
    from paper_2312_15554_amd import abi
    from paper_2312_15554_amd.api import acm_transport_step
    H = I.random_mask(shape, 13, 0.3)
    u = np.zeros((3,) + shape)
    o = O.transport_ls(H, u, (1.0, 0.0, 0.0), 0.0, A0=0.2, eta=0.01, eps=1e-6, max_iter=3000)
    assert o["status"] == "diverged"
    with pytest.raises(abi.AcmError) as e:
        acm_transport_step(dev(H), dev(u, torch.float32), (1.0, 0.0, 0.0), 0.0, A0=0.2,
                           B0=(0.0, 0.0, 0.0), eta=0.01, eps=1e-6, max_iter=3000)
    assert e.value.status == abi.ACM_E_DIVERGED


@pytest.mark.gpu
def test_nan_flow_reports_divergence():
    """A NaN in the advecting flow makes r_1 NaN at once: ACM_E_DIVERGED."""
    require_gpu()
    from paper_2312_15554_amd import abi
    from paper_2312_15554_amd.api import acm_transport_step
    shape = (32, 32, 32)
    H = I.random_mask(shape, 17, 0.3)
    u = np.zeros((3,) + shape)
    pz, py, px = np.argwhere(H == 0)[0]
    u[0, pz, py, px] = np.nan
    with pytest.raises(abi.AcmError) as e:
        acm_transport_step(dev(H), dev(u, torch.float32), (1.0, 0.0, 0.0), 5.0, A0=0.55,
                           B0=(1.0, 0.0, 0.0), eta=0.01, eps=1e-6, max_iter=3000)
    assert e.value.status == abi.ACM_E_DIVERGED


# ------------------------------------------------------------ flux form (Section 3.2, second reading)

@pytest.mark.gpu
@pytest.mark.parametrize("shape", [(16, 16), (8, 24), (16, 24, 32), (16, 32, 32), (8, 16, 64)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("dt", [math.inf, 5e-3])
def test_flux_form_iterates_match_oracle(shape, dtype, dt):
    """Flux form (face fluxes with harmonic-mean diffusivity, forward and
    backward differences): chi after the same LS iterations as the oracle's
    flux form, steady and time-stepped, 2D and 3D (a cube that would take
    the slab form runs the row form here)."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_transport_step
    print(f"flux-form parity shape={shape} dtype={dtype} dt={dt}", flush=True)
    d = len(shape)
    H = I.random_mask(shape, 23, 0.3)
    u = I.random_field((d,) + shape, 29) * (1 - H)
    g = (0.3, 1.0, -0.5)[:d]
    B0 = (0.6, 0.0, 0.1)[:d]
    M, steps = 12, (1 if math.isinf(dt) else 3)
    r = acm_transport_step(dev(H), dev(u, dtype), g, 4.0, A0=1.2, B0=B0, eta=0.05, dt=dt,
                           n_steps=steps, eps=0.0, max_iter=M, form="flux")
    o = O.transport_ls(H, u, g, 4.0, A0=1.2, B0=B0, eta=0.05, dt=dt, n_steps=steps, eps=0.0,
                       max_iter=M, form="flux")
    assert r["stats"]["iters"] == M * steps
    tol = 1e-11 if dtype == torch.float64 else 3e-5
    assert np.abs(host(r["chi"]) - o["chi"]).max() < tol * np.abs(o["chi"]).max()


@pytest.mark.gpu
def test_flux_form_fixed_point_matches_direct_solve_whatever_the_medium():
    """Converged flux-form solves (FP64) with two comparison media equal the
    sparse direct solve of the flux-form equations, which has no A0 in it."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_transport_step
    shape = (8, 16, 16)
    H = I.random_mask(shape, 11, 0.3)
    u = I.random_field((3,) + shape, 12) * (1 - H)
    u = u / np.abs(u).max()
    g = (0.0, 1.0, 0.0)
    ref = O.brute_force_transport(H, u, g, 3.0, eta=0.02, form="flux")
    for A0, B0 in ((1.1, (0.0, 0.0, 0.0)), (2.5, (0.3, -0.2, 0.1))):
        r = acm_transport_step(dev(H), dev(u, torch.float64), g, 3.0, A0=A0, B0=B0, eta=0.02,
                               eps=1e-12, max_iter=40000, form="flux")
        assert r["stats"]["converged"]
        assert np.abs(host(r["chi"]) - ref).max() < 1e-9 * np.abs(ref).max()


@pytest.mark.gpu
def test_flux_form_laminate_flux_and_mass_conservation():
    """Voxel-aligned laminate across x, Pe = 0, g = e_x (FP64): the face flux
    A_f (D+ chi + 1) equals the series conductance 1/mean(1/A) on every face.
    Then, from a random chi with g = 0, backward-Euler steps keep the solute
    mass to rounding."""
    require_gpu()
    from paper_2312_15554_amd.api import acm_effective_props, acm_transport_step
    n = 16
    x = np.arange(n)
    H = np.zeros((8, 8, n), np.uint8)
    H[:, :, x < n // 4] = 1
    eta = 0.05
    A = (1.0 - H) + eta * H
    u = np.zeros((3,) + H.shape)
    r = acm_transport_step(dev(H), dev(u, torch.float64), (1.0, 0.0, 0.0), 0.0, A0=1.0,
                           B0=(0.0, 0.0, 0.0), eta=eta, eps=1e-13, max_iter=40000, form="flux")
    assert r["stats"]["converged"]
    chi = host(r["chi"])
    J = O.face_harmonic_mean(A, 0) * (O.forward_diff(chi, 0) + 1.0)
    assert np.abs(J - 1.0 / np.mean(1.0 / A[0, 0])).max() < 1e-9
    Hm = I.random_mask((8, 16, 16), 3, 0.4)
    chi0 = I.random_field(Hm.shape, 4)
    c = dev(chi0, torch.float64)
    m0 = float(c.sum())
    acm_transport_step(dev(Hm), dev(np.zeros((3,) + Hm.shape), torch.float64), (0.0, 0.0, 0.0),
                       0.0, A0=1.0, B0=(0.0, 0.0, 0.0), eta=0.01, dt=1e-3, n_steps=6, eps=1e-12,
                       max_iter=20000, chi=c, form="flux")
    assert abs(float(c.sum()) - m0) < 1e-12 * float(c.abs().sum())


@pytest.mark.gpu
def test_flux_form_refuses_exact_symbols():
    require_gpu()
    from paper_2312_15554_amd import abi
    from paper_2312_15554_amd.api import acm_transport_step
    H = np.zeros((16, 16), np.uint8)
    H[:4] = 1
    with pytest.raises(abi.AcmError) as e:
        acm_transport_step(dev(H), dev(np.zeros((2, 16, 16)), torch.float32), (1.0, 0.0), 1.0,
                           max_iter=10, derivative="spectral", form="flux")
    assert e.value.status == abi.ACM_E_INVALID
