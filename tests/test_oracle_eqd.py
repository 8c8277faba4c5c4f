"""Pins of the oracle's effective diffusivity (Section 2, eq. D) beyond its
porosity term, from closed forms of the cell problem (eq. unit cell, third
and fourth lines) on plane channels between solid slabs.

* Taylor-Aris dispersion.  A channel of half-width a between slabs, with the
  Poiseuille flow u_x = (a^2 - y^2)/2 (nu = 1, unit body force) and
  g_chi = e_x: chi depends on y only, chi'' = Pe (u_x - ubar) with
  chi'(+-a) = 0, so chi' = Pe y (a^2 - y^2)/6 and
  D*_xx = phi + Pe int (ubar - u_x) chi = phi + int chi'^2
        = phi (1 + 2 Pe^2 a^6 / 945).
  A flipped sign of (ubar - u) lowers D*_xx below phi.
* Layered medium across its layers (Pe = 0, g_chi = e_y), with the
  fictitious diffusivity eta in the solid (Section 3.2, eq. penalization):
  the flux A (1 + chi') is the same in every layer, so
  D*_yy = phi J with J = 1 / (phi + (1 - phi)/eta) (the series mean).
  Dropping the gradient term, or summing it over the whole cell instead of
  the pore, gives phi instead.

Each closed form is checked twice: on fields sampled from the continuum
solution (this pins the formula alone), and on the oracle's own discrete
transport solution (this pins the chain solver + formula as h -> 0).
The last test plants each of those mistakes in a copy of the oracle's
function and checks that a pin fails.
"""
import inspect

import numpy as np
import pytest

from oracle import acm_oracle as O


def _channel(N, w, nx=4):
    """2D cell [y][x]: solid rows [0, w), pore rows [w, N).  The walls of the
    pore channel sit on the voxel faces y = w h and y = 1."""
    H = np.zeros((N, nx), np.uint8)
    H[:w] = 1
    h = 1.0 / N
    y = (np.arange(N) + 0.5) * h
    yc = 0.5 * (1.0 + w * h)
    a = 0.5 * (1.0 - w * h)
    return H, y, yc, a


def _taylor_aris(phi, Pe, a):
    return phi * (1.0 + 2.0 * Pe ** 2 * a ** 6 / 945.0)


def _taylor_fields(N, w, Pe, nx=4):
    """Continuum Taylor-Aris fields sampled at voxel centres: u_x in the pore
    (zero in the solid) and chi^x (its wall value in the solid)."""
    H, y, yc, a = _channel(N, w, nx)
    pore = H[:, 0] == 0
    s = y - yc
    ux = np.where(pore, 0.5 * (a * a - s * s), 0.0)
    chi = np.where(pore, (Pe / 6.0) * (0.5 * a * a * s * s - 0.25 * s ** 4), Pe * a ** 4 / 24.0)
    u = np.zeros((2, N, nx))
    u[0] = ux[:, None]
    chi_x = np.repeat(chi[:, None], nx, axis=1)
    return H, u, chi_x, a


def _laminate_chi(N, w, eta, nx=4):
    """Continuum cross-layer solution (Pe = 0, g_chi = e_y) sampled at voxel
    centres: slope J/eta - 1 in the solid rows, J - 1 in the pore rows."""
    H, y, yc, a = _channel(N, w, nx)
    h = 1.0 / N
    phi = 1.0 - w / N
    J = 1.0 / (phi + (1.0 - phi) / eta)
    ys = w * h
    chi = np.where(y < ys, (J / eta - 1.0) * y, (J / eta - 1.0) * ys + (J - 1.0) * (y - ys))
    return H, np.repeat(chi[:, None], nx, axis=1), phi, J


# ---------------------------------------------------------------- pins

def pin_taylor_aris_sampled(deff):
    """Sampled Taylor-Aris fields: D*_xx -> phi (1 + 2 Pe^2 a^6/945) at
    second order in h (midpoint quadrature of smooth polynomials)."""
    Pe = 200.0
    errs = []
    for N in (32, 64, 128):
        w = N // 4
        H, u, chi_x, a = _taylor_fields(N, w, Pe)
        phi = 1.0 - w / N
        D = deff(H, u, [chi_x, np.zeros_like(chi_x)], Pe)
        exact = _taylor_aris(phi, Pe, a)
        errs.append(abs(D[0, 0] - exact) / exact)
        # the channel is symmetric about its centre line: no cross terms
        assert abs(D[1, 0]) < 1e-12 and abs(D[0, 1]) < 1e-12
    assert errs[-1] < 5e-5, errs
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs


def pin_laminate_sampled(deff):
    """Sampled piecewise-linear cross-layer field.  The central difference is
    exact except at the two pore voxels next to the walls, where the stencil
    reaches one solid voxel; summing over the pore gives exactly
    D*_yy = phi J + (h/2) J (1/eta - 1).  D*_xx (chi^x = 0) is phi."""
    for N, eta in ((32, 0.01), (64, 0.1), (128, 0.5)):
        w = N // 4
        H, chi_y, phi, J = _laminate_chi(N, w, eta)
        u = np.zeros((2, N, chi_y.shape[1]))
        D = deff(H, u, [np.zeros_like(chi_y), chi_y], 0.0)
        h = 1.0 / N
        assert abs(D[1, 1] - (phi * J + 0.5 * h * J * (1.0 / eta - 1.0))) < 1e-12
        assert abs(D[0, 0] - phi) < 1e-14
        assert abs(D[0, 1]) < 1e-14 and abs(D[1, 0]) < 1e-14


def pin_taylor_aris_solved(deff):
    """The oracle's discrete steady cell problem (brute-force solve of the
    LS fixed point) with the exact discrete Poiseuille flow of the same grid:
    D*_xx converges to the Taylor-Aris value of the channel between the voxel
    faces at second order.  (Shifting the flow by a constant does not change
    the dispersion: only u - ubar enters.)"""
    Pe = 200.0
    errs = []
    for N in (32, 64, 128):
        w = N // 4
        H = np.zeros((N, 4), np.uint8)
        H[:w] = 1
        u = np.zeros((2, N, 4))
        u[0] = O.poiseuille_profile(N, w)[:, None]
        chi = O.brute_force_transport(H, u, (1.0, 0.0), Pe, A0=0.55, eta=1e-3)
        D = deff(H, u, [chi], Pe)
        phi = 1.0 - w / N
        exact = _taylor_aris(phi, Pe, 0.5 * (1.0 - w / N))
        errs.append(abs(D[0, 0] - exact) / exact)
    assert errs[-1] < 2e-4, errs
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0, errs


def pin_laminate_solved(deff):
    """Cross-layer diffusion through the oracle's discrete cell problem
    (Pe = 0, eta = 0.5): D*_yy converges to phi J at first order (the central
    stencil reaches across the diffusivity jump at each wall)."""
    eta = 0.5
    errs = []
    for N in (32, 64, 128):
        w = N // 4
        H = np.zeros((N, 4), np.uint8)
        H[:w] = 1
        u = np.zeros((2, N, 4))
        chis = [O.brute_force_transport(H, u, g, 0.0, A0=0.55, eta=eta) for g in ((1.0, 0.0), (0.0, 1.0))]
        D = deff(H, u, chis, 0.0)
        phi = 1.0 - w / N
        J = 1.0 / (phi + (1.0 - phi) / eta)
        errs.append(abs(D[1, 1] - phi * J) / (phi * J))
        assert abs(D[0, 0] - phi) < 1e-12  # along the layers: no obstruction
    assert errs[-1] < 6e-3, errs
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2, errs


PINS = [pin_taylor_aris_sampled, pin_laminate_sampled, pin_taylor_aris_solved, pin_laminate_solved]


@pytest.mark.parametrize("pin", PINS, ids=lambda p: p.__name__)
def test_effective_diffusivity_pins(pin):
    pin(O.effective_diffusivity)


def test_taylor_aris_three_dimensional_cell():
    """The same channel in 3D (slabs normal to y, flow along x): D*_xx is the
    Taylor-Aris value, D*_zz = phi (along the slabs, no flow component)."""
    N, w, Pe = 64, 16, 200.0
    H2, u2, chi2, a = _taylor_fields(N, w, Pe, nx=8)
    H = np.repeat(H2[None], 8, axis=0)
    u = np.zeros((3, 8, N, 8))
    u[0] = u2[0][None]
    chis = [np.repeat(chi2[None], 8, axis=0), np.zeros((8, N, 8)), np.zeros((8, N, 8))]
    D = O.effective_diffusivity(H, u, chis, Pe)
    phi = 1.0 - w / N
    assert abs(D[0, 0] - _taylor_aris(phi, Pe, a)) < 3e-4 * D[0, 0]
    assert abs(D[2, 2] - phi) < 1e-14


MUTATIONS = {
    # flipped sign of (ubar_i - u_i)
    "sign": ("(ubar[i] - u[i])", "(u[i] - ubar[i])"),
    # the gradient term dropped
    "no_grad": ("+ (pore * gc[i]).sum() / Ntot", "+ 0.0"),
    # velocity and gradient terms summed over the whole cell, not the pore
    "whole_cell": ("(pore * (ubar[i] - u[i]) * chi).sum()", "((ubar[i] - u[i]) * chi).sum()"),
    "whole_cell_grad": ("(pore * gc[i]).sum()", "gc[i].sum()"),
}


def _mutant(name):
    src = inspect.getsource(O.effective_diffusivity)
    old, new = MUTATIONS[name]
    assert old in src, f"mutation {name}: pattern not found in the oracle"
    ns = dict(vars(O))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return ns["effective_diffusivity"]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes_fail_a_pin(name):
    """A plausible mistake in eq. D, planted in a copy of the oracle, fails at
    least one of the pins above."""
    f = _mutant(name)
    failed = []
    for pin in PINS:
        try:
            pin(f)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"mutation {name} passes every pin"
