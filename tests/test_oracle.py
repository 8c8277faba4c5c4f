"""Pins for the FP64 oracle, against things other than the oracle itself:
closed forms, real-space stencils, brute-force sparse solves built from
stencils, invariants of the discrete problem and the paper's printed values."""
import json
import math
import os

import numpy as np
import pytest

from oracle import acm_oracle as O
from paper_2312_15554_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- inputs
def test_splitmix64_published_vector():
    ref = json.load(open(os.path.join(GOLD, "splitmix64_seed0.json")))
    rng = I.SplitMix64(ref["seed"])
    got = [rng.next_u64() for _ in ref["outputs_hex"]]
    assert got == [int(h, 16) for h in ref["outputs_hex"]]


def test_disc_rasterisation_matches_lattice_count():
    H = I.centred_disc(64, 0.2)
    cnt = sum(1 for i in range(64) for j in range(64)
              if ((i + 0.5) - 32) ** 2 + ((j + 0.5) - 32) ** 2 <= 12.8 ** 2)
    assert int(H.sum()) == cnt == 524


def test_overlapping_spheres_first_crossing():
    H = I.overlapping_spheres(32, 2.0, 0.5, seed=7)
    por = 1.0 - H.mean()
    assert por <= 0.5 and por > 0.45
    assert np.array_equal(H, I.overlapping_spheres(32, 2.0, 0.5, seed=7))


# ---------------------------------------------------------------- symbols
@pytest.mark.parametrize("shape", [(12, 10), (6, 8, 10)])
def test_symbols_equal_real_space_stencils(shape):
    f = I.random_field(shape, 3)
    s, L = O.symbols(shape)
    F = np.fft.fftn(f)
    gs = O.grad_spectral(F, s)
    gr = O.central_grad(f)
    assert np.allclose(gs, gr, atol=1e-10 * np.abs(gr).max())
    lap_s = np.fft.ifftn(L * F).real
    assert np.allclose(lap_s, O.compact_neg_laplacian(f), atol=1e-9 * np.abs(lap_s).max())


# ---------------------------------------------------------------- Stokes
def _kkt_residual(H, u, q, g, nu=1.0):
    fl = H == 0
    gq = O.central_grad(q)
    mom = np.concatenate([(nu * O.compact_neg_laplacian(u[c]) + gq[c] - g[c])[fl]
                          for c in range(u.shape[0])])
    return np.abs(mom).max(), np.abs(O.central_div(u)).max(), np.abs(u[:, H == 1]).max()


def test_brute_force_reproduces_poiseuille_exactly():
    H = I.slab_cell((16, 16), 4, axis=1)
    u, q = O.brute_force_stokes(H, (1.0, 0.0))
    prof = O.poiseuille_profile(16, 4)
    assert np.abs(u[0] - prof[:, None]).max() < 1e-12
    assert np.abs(u[1]).max() < 1e-12


def test_admm_poiseuille_2d_closed_form_and_darcy():
    N, w = 16, 4
    H = I.slab_cell((N, N), w, axis=1)
    r = O.stokes_admm(H, (1.0, 0.0), eps=1e-10, tau=(20, 10, 30))
    assert r["status"] == "converged"
    prof = O.poiseuille_profile(N, w)
    assert np.abs(r["u"][0] - prof[:, None]).max() < 1e-7 * prof.max()
    K = O.permeability_darcy([r["u"]])
    assert abs(K[0, 0] - prof.sum() / N) < 1e-7 * K[0, 0]
    assert abs(K[0, 1]) < 1e-9
    # flow across the slabs is blocked: K_yy = 0
    r2 = O.stokes_admm(H, (0.0, 1.0), eps=1e-10, tau=(20, 10, 30))
    assert abs(O.permeability_darcy([r2["u"]])[0, 1]) < 1e-9


def test_admm_poiseuille_3d_slab_all_directions():
    shape = (8, 12, 8)  # [z][y][x]; slab normal to y
    H = I.slab_cell(shape, 3, axis=1)
    prof = O.poiseuille_profile(12, 3)
    us = []
    for g in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        r = O.stokes_admm(H, g, eps=1e-10)
        assert r["status"] == "converged"
        us.append(r["u"])
    assert np.abs(us[0][0] - prof[None, :, None]).max() < 1e-7 * prof.max()
    assert np.abs(us[2][2] - prof[None, :, None]).max() < 1e-7 * prof.max()
    K = O.permeability_darcy(us)
    kx = prof.sum() / 12
    assert np.allclose(np.diag(K), [kx, 0.0, kx], atol=1e-7 * kx)


@pytest.mark.parametrize("shape,g,seed", [((12, 12), (1.0, 0.5), 3), ((4, 6, 8), (0.3, 1.0, 0.2), 5)])
def test_admm_converges_to_brute_force_kkt(shape, g, seed):
    H = I.random_mask(shape, seed, 0.3)
    ub, qb = O.brute_force_stokes(H, g)
    k = _kkt_residual(H, ub, qb, g)
    assert max(k) < 1e-9
    r = O.stokes_admm(H, g, eps=1e-13, max_iter=100000)
    assert r["status"] == "converged"
    assert np.abs(r["u"] - ub).max() < 1e-7 * np.abs(ub).max()


def test_stokes_invariants_random_cell():
    H = I.overlapping_spheres((8, 8, 8), 1.5, 0.55, seed=11)
    us = []
    eps = 1e-8
    for g in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        r = O.stokes_admm(H, g, eps=eps)
        assert r["status"] == "converged"
        u = r["u"]
        # constraints hold to the ADMM tolerance
        assert np.linalg.norm(O.central_div(u)) <= r["tol_p"][1] * 1.0001
        assert np.linalg.norm(u[:, H == 1]) <= 10 * math.sqrt(u.size) * eps + 1e-6 * np.linalg.norm(u)
        us.append(u)
    Kd = O.permeability_darcy(us)
    Ke = O.permeability_energy(us)
    assert np.allclose(Kd, Ke, rtol=1e-4, atol=1e-8 * np.abs(Kd).max())
    assert np.allclose(Kd, Kd.T, atol=1e-4 * np.abs(Kd).max())
    assert np.all(np.linalg.eigvalsh(0.5 * (Kd + Kd.T)) > 0)


def test_fixed_point_independent_of_penalty_schedule():
    H = I.random_mask((10, 10), 9, 0.35)
    g = (1.0, 0.0)
    r1 = O.stokes_admm(H, g, eps=1e-12)
    r2 = O.stokes_admm(H, g, alpha=13.0, beta=40.0, b=7.0, tau=(20, 10, 30), eps=1e-12)
    assert r1["status"] == r2["status"] == "converged"
    assert abs(r1["iters"] - r2["iters"]) > 0
    assert np.abs(r1["u"] - r2["u"]).max() < 1e-7 * np.abs(r1["u"]).max()


def test_adaptive_penalties_need_fewer_iterations():
    # Section 4.1: varying the penalties converges in fewer iterations than
    # keeping them fixed (starting from a poor fixed choice).
    H = I.centred_disc(32)
    kw = dict(alpha=3200.0, beta=3200.0, b=3200.0, eps=1e-5, tau=(20, 10, 30), max_iter=20000)
    ra = O.stokes_admm(H, (1, 0), adaptive=True, **kw)
    rf = O.stokes_admm(H, (1, 0), adaptive=False, **kw)
    assert ra["status"] == rf["status"] == "converged"
    assert ra["iters"] < rf["iters"]


def test_c1_disc_matches_dilute_cylinder_array():
    # Hasimoto (1959) leading-order permeability of a square array of
    # cylinders at solid fraction c: k = (-0.5 ln c - 0.738 + c) / (4 pi).
    H = I.centred_disc(64)
    r = O.stokes_admm(H, (1.0, 0.0), eps=1e-5, tau=(20, 10, 30))
    c = H.mean()
    k_ref = (-0.5 * math.log(c) - 0.738 + c) / (4 * math.pi)
    k = O.permeability_darcy([r["u"]])[0, 0]
    assert abs(k - k_ref) < 0.05 * k_ref


def test_warm_start_from_solution_converges_immediately():
    H = I.random_mask((10, 10), 4, 0.3)
    g = (1.0, 0.3)
    r = O.stokes_admm(H, g, eps=1e-12)
    r2 = O.stokes_admm(H, g, eps=1e-9, u_init=r["u"], q_init=r["q"])
    assert r2["status"] == "converged" and r2["iters"] < 5
    assert np.abs(r2["u"] - r["u"]).max() < 1e-7 * np.abs(r["u"]).max()


# ---------------------------------------------------------------- transport
def test_diffusion_mode_decay_closed_form():
    shape = (16, 16)
    H = np.zeros(shape, np.uint8)
    u = np.zeros((2,) + shape)
    y, x = np.meshgrid((np.arange(16) + 0.5) / 16, (np.arange(16) + 0.5) / 16, indexing="ij")
    mode = (2, 1)
    chi0 = np.cos(2 * np.pi * (mode[0] * x + mode[1] * y))
    dt, n = 2e-3, 5
    r = O.transport_ls(H, u, (0.0, 0.0), 0.0, A0=0.55, B0=(0.0, 0.0), eps=1e-12,
                       dt=dt, n_steps=n, chi_init=chi0)
    amp = O.diffusion_mode_amplitude(shape, mode, dt, n, 0.55)
    assert r["status"] == "converged"
    assert np.abs(r["chi"] - amp * chi0).max() < 1e-9
    # the brute-force time step reproduces the same closed form
    c = chi0
    for _ in range(n):
        c = O.brute_force_transport(H, u, (0.0, 0.0), 0.0, A0=0.55, dt=dt, chi_prev=c)
    assert np.abs(c - amp * chi0).max() < 1e-12


def test_transport_homogeneous_cell_gives_identity():
    shape = (8, 8, 8)
    H = np.zeros(shape, np.uint8)
    u = np.zeros((3,) + shape)
    r = O.transport_ls(H, u, (1.0, 0.0, 0.0), 0.0, B0=(1.0, 0.0, 0.0), eps=1e-12)
    assert np.abs(r["chi"]).max() < 1e-12
    D = O.effective_diffusivity(H, u, [r["chi"]], 0.0)
    assert np.allclose(D[:, 0], [1.0, 0.0, 0.0])


def _flow(H, g):
    u, _ = O.brute_force_stokes(H, g)
    return u / np.abs(u).max()


@pytest.mark.parametrize("B0", [(0.0, 0.0), (1.0, 0.0)])
def test_ls_steady_matches_brute_force(B0):
    H = I.random_mask((12, 12), 21, 0.3)
    u = _flow(H, (1.0, 0.0))
    g = (1.0, 0.0)
    chi_bf = O.brute_force_transport(H, u, g, 5.0, A0=0.55, eta=0.01)
    r = O.transport_ls(H, u, g, 5.0, A0=0.55, B0=B0, eta=0.01, eps=1e-13, max_iter=20000)
    assert r["status"] == "converged"
    assert np.abs(r["chi"] - chi_bf).max() < 1e-8 * np.abs(chi_bf).max()
    assert abs(r["chi"].mean()) < 1e-14


def test_ls_time_steps_match_brute_force_and_conserve_mass_trend():
    H = I.random_mask((4, 6, 8), 8, 0.3)
    u = _flow(H, (1.0, 0.0, 0.0))
    g = (0.0, 1.0, 0.0)
    dt, n = 5e-3, 3
    r = O.transport_ls(H, u, g, 3.0, A0=0.55, B0=(0.5, 0.0, 0.0), eps=1e-13, dt=dt, n_steps=n)
    c = np.zeros(H.shape)
    for _ in range(n):
        c = O.brute_force_transport(H, u, g, 3.0, A0=0.55, dt=dt, chi_prev=c)
    assert r["status"] == "converged"
    assert np.abs(r["chi"] - c).max() < 1e-8 * np.abs(c).max()


def test_effective_diffusivity_nonsymmetric_with_flow():
    # eq. D: with Pe > 0 the effective diffusivity need not be symmetric.
    H = I.overlapping_spheres((16, 16), 2.5, 0.6, seed=3)
    u = _flow(H, (1.0, 0.3))
    chis = [O.transport_ls(H, u, g, 20.0, B0=(0.0, 0.0), eps=1e-10)["chi"] for g in [(1, 0), (0, 1)]]
    D = O.effective_diffusivity(H, u, chis, 20.0)
    assert abs(D[0, 1] - D[1, 0]) > 1e-3 * abs(D).max()
    D0 = O.effective_diffusivity(H, u, chis, 0.0)
    assert np.all(np.isfinite(D0))


def test_paper_parameters_fixture():
    p = json.load(open(os.path.join(GOLD, "paper_parameters.json")))
    assert p["comparison_medium_A0"]["value"] == 0.55
    assert p["adaptive_tau_model_geometry"]["value"] == [20, 10, 30]
    assert p["adaptive_tau_random_geometry"]["value"] == [5, 10, 5]


@pytest.mark.parametrize("shape", [(12, 8), (8, 12, 16)])
def test_spectral_symbols_differentiate_fourier_modes_exactly(shape):
    """The exact-FFT symbols (kind "spectral", the alternative to eq. fft_app
    the paper compares in Section 4) give the calculus derivatives of a
    resolved Fourier mode: each d/dx_c and the Laplacian of sin(2 pi m.x).
    The central symbols of eq. fft_app miss them at second order in h."""
    nd = len(shape)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    m = [1, 2, 3][:nd]  # per numpy axis, below n/2
    phase = 2 * np.pi * sum(m[a] * grids[a] for a in range(nd))
    f = np.sin(phase)
    fh = np.fft.fftn(f)
    s, L = O.symbols(shape, "spectral")
    for c in range(nd):
        ax = nd - 1 - c
        d = np.real(np.fft.ifftn(1j * s[c] * fh))
        assert np.abs(d - 2 * np.pi * m[ax] * np.cos(phase)).max() < 1e-10
    lap = np.real(np.fft.ifftn(-L * fh))
    k2 = (2 * np.pi) ** 2 * sum(mm * mm for mm in m)
    assert np.abs(lap + k2 * f).max() < 1e-9 * k2
    _, Lc = O.symbols(shape, "central")
    assert np.abs(np.real(np.fft.ifftn(-Lc * fh)) - lap).max() > 1e-3 * k2


def test_spectral_diffusion_mode_decay_closed_form():
    """Pure diffusion of one Fourier mode with the exact symbols: each
    backward-Euler step divides it by 1 + dt |k|^2, |k| = 2 pi |m|."""
    shape = (16, 16)
    H = np.zeros(shape, np.uint8)
    u = np.zeros((2,) + shape)
    y, x = np.meshgrid((np.arange(16) + 0.5) / 16, (np.arange(16) + 0.5) / 16, indexing="ij")
    mode = (2, 1)
    chi0 = np.cos(2 * np.pi * (mode[0] * x + mode[1] * y))
    dt, n = 2e-3, 5
    r = O.transport_ls(H, u, (0.0, 0.0), 0.0, A0=0.55, B0=(0.0, 0.0), eps=1e-12,
                       dt=dt, n_steps=n, chi_init=chi0, derivative="spectral")
    amp = (1.0 + dt * (2 * np.pi) ** 2 * (mode[0] ** 2 + mode[1] ** 2)) ** (-n)
    assert r["status"] == "converged"
    assert np.abs(r["chi"] - amp * chi0).max() < 1e-9


def test_spectral_admm_satisfies_the_spectral_stokes_equations():
    """ADMM with the exact symbols converges to a field that satisfies the
    Stokes equations with exact spectral derivatives (written here with
    numpy's own wavenumbers): divergence-free, momentum balance in the pore,
    no velocity in the solid."""
    shape = (16, 16)
    H = I.random_mask(shape, 3, 0.3)
    g = (1.0, 0.3)
    r = O.stokes_admm(H, g, eps=1e-10, tau=(20, 10, 30), derivative="spectral")
    assert r["status"] == "converged"
    u, q = r["u"], r["q"]
    ky, kx = np.meshgrid(2 * np.pi * np.fft.fftfreq(16, 1 / 16), 2 * np.pi * np.fft.fftfreq(16, 1 / 16),
                         indexing="ij")
    k1 = [kx.copy(), ky.copy()]
    for kk in k1:  # first derivatives drop the Nyquist mode of a real field
        kk[np.isclose(np.abs(kk), np.pi * 16)] = 0.0
    k2 = kx ** 2 + ky ** 2
    uh = [np.fft.fft2(u[c]) for c in range(2)]
    div = np.real(np.fft.ifft2(1j * k1[0] * uh[0] + 1j * k1[1] * uh[1]))
    scale = np.abs(u).max() * 2 * np.pi * 16
    assert np.abs(div).max() < 1e-6 * scale
    qh = np.fft.fft2(q)
    pore = H == 0
    for c in range(2):
        mom = g[c] - np.real(np.fft.ifft2(1j * k1[c] * qh)) - np.real(np.fft.ifft2(k2 * uh[c]))
        assert np.abs(mom[pore]).max() < 1e-5 * max(1.0, np.abs(g).max())
        assert np.abs(u[c][~pore]).max() < 1e-5 * np.abs(u).max()  # ADMM constraint at eps
