"""Pins for the flux form of the transport discretisation in the oracle (the
second reading of the Section 3.2 scheme: forward-difference gradient,
face harmonic-mean diffusivity, backward-difference divergence).  Each pin
comes from outside the oracle's LS iteration: a sparse direct solve built
from difference matrices, the closed-form flux through a laminate, the
closed-form decay of a Fourier mode, exact conservation of solute mass, and
the independence of the fixed point from the comparison medium."""
import math

import numpy as np
import pytest

from oracle import acm_oracle as O
from paper_2312_15554_amd import inputs as I


def _flow(H, seed):
    u = I.random_field((H.ndim,) + H.shape, seed) * (1 - H)
    return u / np.abs(u).max()


@pytest.mark.parametrize("shape", [(12, 16), (6, 8, 10)])
@pytest.mark.parametrize("dt", [math.inf, 0.01])
def test_flux_form_fixed_point_equals_direct_solve(shape, dt):
    """LS iteration (flux form) to eps = 1e-12 equals the sparse direct solve
    of the flux-form equations, with flow (Pe = 4) and a solid phase."""
    H = I.random_mask(shape, 5, 0.3)
    u = _flow(H, 7)
    g = (1.0, -0.5, 0.25)[:len(shape)]
    chi0 = I.random_field(shape, 9) * 0.1
    kw = dict(A0=1.2, B0=(0.5, 0.0, 0.0)[:len(shape)], eta=0.05)
    r = O.transport_ls(H, u, g, 4.0, eps=1e-12, max_iter=20000, dt=dt, n_steps=1,
                       chi_init=None if math.isinf(dt) else chi0, form="flux", **kw)
    assert r["status"] == "converged"
    ref = O.brute_force_transport(H, u, g, 4.0, A0=1.2, eta=0.05, dt=dt,
                                  chi_prev=None if math.isinf(dt) else chi0, form="flux")
    assert np.abs(r["chi"] - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_flux_form_fixed_point_is_free_of_the_comparison_medium():
    """Two comparison media (A0, B0) give the same flux-form fixed point; the
    central form's fixed point moves with A0 by its O(h^2) A0 (L - |s|^2)
    term, so this pin separates the two readings."""
    shape = (10, 12, 8)
    H = I.random_mask(shape, 11, 0.3)
    u = _flow(H, 12)
    g = (0.0, 1.0, 0.0)
    sols = {}
    for form in ("flux", "central"):
        for A0, B0 in ((1.1, (0.0, 0.0, 0.0)), (2.5, (0.3, -0.2, 0.1))):
            r = O.transport_ls(H, u, g, 3.0, A0=A0, B0=B0, eta=0.02, eps=1e-12, max_iter=40000,
                               form=form)
            assert r["status"] == "converged", (form, A0)
            sols[(form, A0)] = r["chi"]
    scale = np.abs(sols[("flux", 1.1)]).max()
    assert np.abs(sols[("flux", 1.1)] - sols[("flux", 2.5)]).max() < 1e-9 * scale
    assert np.abs(sols[("central", 1.1)] - sols[("central", 2.5)]).max() > 1e-3 * scale


@pytest.mark.parametrize("n", [8, 16])
def test_flux_through_a_laminate_is_the_harmonic_mean(n):
    """Layers normal to x (H depends on x only), Pe = 0, g = e_x: the
    discrete flux J = A_f (D+ chi + 1) is the same on every face and equals
    the series conductance of the voxel-aligned laminate, 1 / mean(1 / A)
    over the voxels (the exact flux of the continuous layered medium, the
    harmonic-mean bound).  The central form gives another flux, so the pin
    fixes the face coefficient and the forward/backward pairing."""
    x = np.arange(n)
    H = np.zeros((4, n), np.uint8)
    H[:, (x % n) < n // 4] = 1
    eta = 0.05
    A = (1.0 - H) + eta * H
    u = np.zeros((2, 4, n))
    r = O.transport_ls(H, u, (1.0, 0.0), 0.0, A0=1.0, eta=eta, eps=1e-13, max_iter=20000, form="flux")
    assert r["status"] == "converged"
    Af = O.face_harmonic_mean(A, 0)
    J = Af * (O.forward_diff(r["chi"], 0) + 1.0)
    J_exact = 1.0 / np.mean(1.0 / A[0])
    assert np.abs(J - J_exact).max() < 1e-9
    rc = O.transport_ls(H, u, (1.0, 0.0), 0.0, A0=1.0, eta=eta, eps=1e-13, max_iter=20000)
    Jc = Af * (O.forward_diff(rc["chi"], 0) + 1.0)
    assert np.abs(Jc - J_exact).max() > 1e-3


def test_flux_form_mode_decay_closed_form():
    """H = 0, Pe = 0: a cosine mode decays by (1 + dt L(m))^(-n) after n
    backward-Euler steps in the flux form, whatever A0 (the central form
    decays with (1 - A0)|s|^2 + A0 L instead)."""
    shape = (16, 24)
    mode = (2, 3)
    y, x = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    chi0 = np.cos(2 * np.pi * (mode[0] * x / shape[1] + mode[1] * y / shape[0]))
    H = np.zeros(shape, np.uint8)
    u = np.zeros((2,) + shape)
    for A0 in (0.7, 1.6):
        r = O.transport_ls(H, u, (0.0, 0.0), 0.0, A0=A0, eps=1e-13, max_iter=5000, dt=2e-3,
                           n_steps=5, chi_init=chi0, form="flux")
        amp = O.diffusion_mode_amplitude(shape, mode, 2e-3, 5, A0, form="flux")
        assert np.abs(r["chi"] - amp * chi0).max() < 1e-11
        amp_c = O.diffusion_mode_amplitude(shape, mode, 2e-3, 5, A0)
        assert abs(amp - amp_c) > 1e-4


def test_flux_form_conserves_mass_under_pure_diffusion():
    """Pe = 0 and g = 0 with a solid phase (eta = 0.01): backward-Euler steps
    of the flux form keep the solute mass h^d sum chi to rounding (the
    backward differences of the face fluxes telescope)."""
    shape = (8, 10, 12)
    H = I.random_mask(shape, 3, 0.4)
    u = np.zeros((3,) + shape)
    chi0 = I.random_field(shape, 4)
    m0 = O.solute_mass(chi0)
    r = O.transport_ls(H, u, (0.0, 0.0, 0.0), 0.0, A0=1.0, eta=0.01, eps=1e-12, max_iter=20000,
                       dt=1e-3, n_steps=6, chi_init=chi0, form="flux")
    assert r["status"] == "converged"
    assert abs(O.solute_mass(r["chi"]) - m0) < 1e-12 * np.abs(chi0).mean()


def test_flux_form_pins_catch_plausible_mistakes(monkeypatch):
    """Mutated copies of the face coefficient (arithmetic mean instead of
    harmonic) and of the divergence (forward instead of backward) fail the
    laminate pin or the direct-solve pin."""
    harmonic = O.face_harmonic_mean
    monkeypatch.setattr(O, "face_harmonic_mean",
                        lambda A, c: 0.5 * (A + np.roll(A, -1, axis=A.ndim - 1 - c)))
    with pytest.raises(AssertionError):
        test_flux_through_a_laminate_is_the_harmonic_mean(8)
    monkeypatch.setattr(O, "face_harmonic_mean", harmonic)
    monkeypatch.setattr(O, "backward_diff", O.forward_diff)
    H = I.random_mask((12, 16), 5, 0.3)
    u = _flow(H, 7)
    r = O.transport_ls(H, u, (1.0, -0.5), 4.0, A0=1.2, eta=0.05, eps=1e-12, max_iter=20000,
                       form="flux")
    monkeypatch.undo()
    ref = O.brute_force_transport(H, u, (1.0, -0.5), 4.0, A0=1.2, eta=0.05, form="flux")
    assert r["status"] != "converged" or np.abs(r["chi"] - ref).max() > 1e-6 * np.abs(ref).max()
