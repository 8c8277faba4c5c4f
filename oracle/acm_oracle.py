"""FP64 CPU oracle for the ACM unit-cell solvers (Karimi & Bhattacharya,
"Accelerated Computational Micromechanics for Reactive Flow in Porous Media").

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the HIP path (no kernels, headers, tables or helpers) and imports nothing
from it.

Everything here is plain NumPy/SciPy in float64 and follows the paper's steps in
its own order:

* Stokes flow: augmented Lagrangian + ADMM, Section 3.1 (eq. Lagrangian with
  auxiliary variable, Steps 1-4, eq. FFT step1), with the adaptive penalties
  of Section 4.1 (eq. varying algorithm).
* Solute transport: fictitious-diffusivity penalisation and Lippmann-Schwinger
  iteration, Section 3.2 (eq. penalization, eq. iter, eq. fft_solute,
  eq. tol_solute), with the central-difference symbols of eq. fft_app.
* Effective properties: eq. K and eq. D of Section 2.
* Brute-force sparse direct solves of the same discrete equations, built from
  real-space stencils, for cross-checking the iterations on tiny grids.

Discretisation conventions (readings of the paper, also used by the HIP path):

* Grid N_1 x ... x N_d on the unit cell, h_j = 1/N_j, fields are numpy arrays
  indexed [z][y][x] (x fastest); vector component c (0=x, 1=y, 2=z) lives on
  numpy axis ndim-1-c.  Vector fields have shape (d, *grid).
* First derivatives use the central-difference symbol s_j = sin(2 pi m_j/N_j)/h_j
  (eq. fft_app, first line); second derivatives use the compact symbol
  L = sum_j 4 sin^2(pi m_j/N_j)/h_j^2 (eq. fft_app, second line).  Both Stokes
  and transport use these symbols.
* Forward DFT unnormalised; the DFT of a constant g is N_tot * g at k = 0.
* Norms are Euclidean over grid values; n in sqrt(n) counts scalar entries.
* Stokes converges when all six residuals are within tolerance; tolerances of
  constraints 2 and 3 follow the pattern the paper gives for constraint 1,
  with multipliers (lambda, q, a) for constraints (1, 2, 3).
* Penalties updated after Step 4 of iteration n are used from iteration n+1;
  dual residuals use the penalties of iteration n.
* Transport: r_2's tolerance is sqrt(n) eps with n = d * N_tot; steady solves
  fix the k = 0 mode to zero (mean-zero chi); time-dependent solves use
  backward Euler with unit capacity over the whole cell.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

WORKERS = max(1, min(os.cpu_count() or 1, 16))


def set_workers(n: int) -> None:
    """Thread count used by scipy.fft inside the oracle."""
    global WORKERS
    WORKERS = max(1, int(n))


def _fft(f):
    return sfft.fftn(f, workers=WORKERS)


def _ifft(F):
    return sfft.ifftn(F, workers=WORKERS).real


# ---------------------------------------------------------------------------
# Symbols (Section 3.2, eq. fft_app)
# ---------------------------------------------------------------------------

def symbols(shape, kind="central"):
    """First-derivative symbols s_c and Laplacian symbol L on the unit cell.

    kind "central" (the paper's scheme, Section 3.3): s_c = sin(theta_c)/h_c,
    the symbol of the central difference, and the compact Laplacian
    L = sum_c 4 sin^2(theta_c/2)/h_c^2.  kind "spectral" (the exact-FFT
    alternative the paper compares against in Section 4): s_c = theta_c/h_c =
    2 pi m_c and L = sum_c (2 pi m_c)^2, with m_c the signed wavenumber.
    Returns (s, L): s is a list with one broadcastable array per vector
    component c (0=x on the last numpy axis).  s_c vanishes at the Nyquist
    index in both (sin(pi) = 0; a real field has no odd Nyquist derivative).
    """
    if kind not in ("central", "spectral"):
        raise ValueError("kind must be 'central' or 'spectral'")
    nd = len(shape)
    s = []
    L = np.zeros([1] * nd)
    for c in range(nd):
        ax = nd - 1 - c
        n = shape[ax]
        m = np.fft.fftfreq(n, d=1.0 / n)
        theta = 2.0 * np.pi * m / n
        if kind == "central":
            sc = np.sin(theta) * n
            lc = 4.0 * np.sin(theta / 2.0) ** 2 * n * n
        else:
            sc = theta * n
            lc = (theta * n) ** 2
        if n % 2 == 0:
            sc[np.abs(m) == n // 2] = 0.0
        bshape = [1] * nd
        bshape[ax] = n
        s.append(sc.reshape(bshape))
        L = L + lc.reshape(bshape)
    return s, L


def grad_spectral(f_hat, s):
    """Central-difference gradient of a scalar given its spectrum."""
    return np.stack([_ifft(1j * sc * f_hat) for sc in s])


def div_spectral_hat(v_hat, s):
    """Spectrum of the central-difference divergence of a vector spectrum."""
    return sum(1j * s[c] * v_hat[c] for c in range(len(s)))


# Real-space stencils (used by invariants and brute-force solves) -----------

def central_grad(f):
    """(f(x+h e_c) - f(x-h e_c)) / (2 h_c) for every component c, periodic."""
    nd = f.ndim
    out = []
    for c in range(nd):
        ax = nd - 1 - c
        n = f.shape[ax]
        out.append((np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) * (n / 2.0))
    return np.stack(out)


def central_div(v):
    nd = v.shape[0]
    tot = 0.0
    for c in range(nd):
        ax = nd - 1 - c
        n = v.shape[1 + ax]
        tot = tot + (np.roll(v[c], -1, axis=ax) - np.roll(v[c], 1, axis=ax)) * (n / 2.0)
    return tot


def compact_neg_laplacian(f):
    """-Delta_h f with the 3-point (2d+1 point) compact stencil, periodic."""
    nd = f.ndim
    out = 0.0
    for c in range(nd):
        ax = nd - 1 - c
        n = f.shape[ax]
        out = out + (2.0 * f - np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) * (n * n)
    return out


# ---------------------------------------------------------------------------
# Stokes flow by ADMM (Section 3.1, Steps 1-4; Section 4.1 adaptive penalties)
# ---------------------------------------------------------------------------

def default_penalty(shape, nu=1.0):
    """Initial penalties (the paper leaves them unstated): psi0 = nu/h for
    alpha, beta and b, floor psi_min = 1e-3 psi0."""
    n = max(shape)
    p0 = nu * n
    return dict(alpha=p0, beta=p0, b=p0, psi_min=(1e-3 * p0,) * 3)


def stokes_admm(H, g, nu=1.0, alpha=None, beta=None, b=None,
                phi=(1.1, 1.1, 1.1), tau=(5.0, 10.0, 5.0), psi_min=None,
                adaptive=True, eps=1e-6, max_iter=100000,
                u_init=None, q_init=None, history=False, derivative="central"):
    """Solve the unit-cell Stokes problem (eq. unit cell, first two lines) by
    the paper's ADMM on the extended domain.

    H: solid indicator (1 solid, 0 pore), numpy shape [z][y][x] or [y][x].
    g: body force / imposed pressure gradient g_p, length d (x, y[, z]).
    Returns a dict with the final iterate X^{n+1} = (u, ut, q, a, lam), the
    iteration count, the status ('converged' | 'not_converged' | 'diverged'),
    the last residuals, tolerances and penalties.

    Warm start (u_init/q_init given): u0 = ut0 = (1-H) u_init, q0 = q_init,
    a0 = lam0 = H (g - grad q0 + nu Delta u0), the reaction the fixed point
    carries in the solid.
    """
    H = np.asarray(H)
    shape = H.shape
    d = len(shape)
    Ntot = H.size
    Hf = H.astype(np.float64)
    s, L = symbols(shape, derivative)
    pen = default_penalty(shape, nu)
    alpha = pen["alpha"] if alpha is None else float(alpha)
    beta = pen["beta"] if beta is None else float(beta)
    b = pen["b"] if b is None else float(b)
    psi = [alpha, beta, b]
    psi_min = list(pen["psi_min"] if psi_min is None else psi_min)
    gvec = [float(g[c]) for c in range(d)]

    # --- initial state X^0
    if u_init is None:
        u = np.zeros((d,) + shape)
    else:
        u = (1.0 - Hf) * np.asarray(u_init, dtype=np.float64)
    ut = u.copy()
    q = np.zeros(shape) if q_init is None else np.asarray(q_init, dtype=np.float64).copy()
    if u_init is None and q_init is None:
        a = np.zeros((d,) + shape)
        lam = np.zeros((d,) + shape)
    else:
        q_hat0 = _fft(q)
        grad_q = grad_spectral(q_hat0, s)
        lap_u = np.stack([-_ifft(L * _fft(u[c])) for c in range(d)])
        reaction = np.stack([gvec[c] - grad_q[c] + nu * lap_u[c] for c in range(d)])
        a = Hf * reaction
        lam = a.copy()
    u_hat = np.stack([_fft(u[c]) for c in range(d)])
    divu = _ifft(div_spectral_hat(u_hat, s))

    # Step-1 operator pieces: M(k) = (nu L + b) I + beta s s^T
    S = np.stack(np.broadcast_arrays(*s), axis=-1)  # (*grid, d)
    eye = np.eye(d)

    n_vec = d * Ntot
    n_sca = Ntot
    sq = (math.sqrt(n_vec), math.sqrt(n_sca), math.sqrt(n_vec))
    status = "not_converged"
    hist = []
    it = 0
    rp = rd = tp = td = [np.nan] * 3
    rsum_min = math.inf
    for it in range(1, max_iter + 1):
        al, be, bb = psi
        # Step 1: stationarity in u (eq. step1por solved in Fourier, eq. FFT step1)
        rhs = np.stack([_fft(gvec[c] * np.ones(shape) - a[c] + bb * ut[c]) for c in range(d)])
        q_hat = _fft(q)
        rhs = rhs - np.stack([1j * s[c] * q_hat for c in range(d)])
        M = (nu * L + bb)[..., None, None] * eye + be * S[..., :, None] * S[..., None, :]
        rhs_last = np.moveaxis(rhs, 0, -1)
        uh = np.linalg.solve(M, rhs_last[..., None])[..., 0]
        u_hat_new = np.moveaxis(uh, -1, 0)
        u_new = np.stack([_ifft(u_hat_new[c]) for c in range(d)])
        # Step 2: stationarity in ut (eq. u_tilde), pointwise
        ut_new = (a + bb * u_new - Hf * lam) / (bb + al * Hf)
        # Step 3: multiplier updates (eq. Lagrange-multipliers), pointwise
        divu_new = _ifft(div_spectral_hat(u_hat_new, s))
        q_new = q - be * divu_new
        a_new = a + bb * (u_new - ut_new)
        lam_new = lam + al * (Hf * ut_new)
        # Step 4: residuals (eq. constrains) and tolerances
        rp = [np.linalg.norm(Hf * ut_new),
              np.linalg.norm(divu_new),
              np.linalg.norm(u_new - ut_new)]
        rd = [al * np.linalg.norm(Hf * (ut_new - ut)),
              be * np.linalg.norm(divu_new - divu),
              bb * np.linalg.norm(u_new - u)]
        mu = [np.linalg.norm(lam_new), np.linalg.norm(q_new), np.linalg.norm(a_new)]
        tp = [sq[k] * eps + eps * max(rp[k], mu[k]) for k in range(3)]
        td = [sq[k] * eps + eps * mu[k] for k in range(3)]
        u, ut, q, a, lam, divu = u_new, ut_new, q_new, a_new, lam_new, divu_new
        if history:
            hist.append(dict(rp=list(rp), rd=list(rd), tp=list(tp), td=list(td), psi=list(psi)))
        # divergence: a non-finite residual, or the sum of the six grown a
        # millionfold over its smallest value so far
        rsum = sum(rp) + sum(rd)
        rsum_min = min(rsum_min, rsum)
        if not all(np.isfinite(rp + rd)) or (it > 5 and rsum > 1e6 * rsum_min):
            status = "diverged"
            break
        if all(rp[k] <= tp[k] and rd[k] <= td[k] for k in range(3)):
            status = "converged"
            break
        # adaptive penalties (eq. varying algorithm), pairs alpha<->1, beta<->2, b<->3
        if adaptive:
            for k in range(3):
                if rp[k] > tau[k] * rd[k]:
                    psi[k] = phi[k] * psi[k]
                elif rd[k] > tau[k] * rp[k]:
                    psi[k] = max(psi[k] / phi[k], psi_min[k])
    return dict(u=u, ut=ut, q=q, a=a, lam=lam, iters=it, status=status,
                r_p=rp, r_d=rd, tol_p=tp, tol_d=td, psi=list(psi), history=hist)


# ---------------------------------------------------------------------------
# Solute transport by the Lippmann-Schwinger iteration (Section 3.2)
# ---------------------------------------------------------------------------

def pore_mean_velocity(H, u):
    """u-bar = (1/|Y_p|) integral over the pore of u (Section 2)."""
    pore = 1.0 - np.asarray(H, dtype=np.float64)
    return np.array([(pore * u[c]).sum() / pore.sum() for c in range(u.shape[0])])


def face_harmonic_mean(A, c):
    """Diffusivity on the face between x and x + h e_c: the harmonic mean
    2 A(x) A(x + h e_c) / (A(x) + A(x + h e_c)), the coefficient of a flux
    through two voxels in series."""
    ax = A.ndim - 1 - c
    Ap = np.roll(A, -1, axis=ax)
    return 2.0 * A * Ap / (A + Ap)


def forward_diff(f, c):
    """(f(x + h e_c) - f(x)) / h_c, periodic."""
    ax = f.ndim - 1 - c
    return (np.roll(f, -1, axis=ax) - f) * f.shape[ax]


def backward_diff(f, c):
    """(f(x) - f(x - h e_c)) / h_c, periodic."""
    ax = f.ndim - 1 - c
    return (f - np.roll(f, 1, axis=ax)) * f.shape[ax]


def transport_ls(H, u, g, Pe, A0=0.55, B0=None, eta=0.01, diffusivity=1.0,
                 eps=1e-6, max_iter=100000, dt=math.inf, n_steps=1,
                 chi_init=None, history=False, derivative="central", form="central"):
    """Penalised advection-diffusion (eq. penalization) by the LS iteration
    (eq. iter, solved in Fourier by eq. fft_solute with the symbols of
    eq. fft_app; derivative="spectral" takes the exact symbols instead).

    A = diffusivity (1-H) + eta H, B = Pe (1-H) u, calF = Pe (1-H) ubar . g.
    dt = inf: the paper's steady cell problem (one solve, chi-hat(0) = 0).
    finite dt: n_steps backward-Euler steps of d chi/dt + [operator] = calF,
    each solved by the LS iteration with comparison symbol
    1/dt + A0 L + i B0 . s.
    form="central" (the literal reading): the diffusive term of the residual
    is the central divergence of (A - A0)(grad_c chi + g), so the fixed point
    keeps an O(h^2) term A0 (L - |s|^2) chi.  form="flux": the diffusive flux
    through the face between x and x + h e_c is A_f (D+_c chi + g_c) with the
    face's harmonic-mean diffusivity A_f and the forward difference D+, and
    its divergence is the backward difference D-; since -D-.(A0 D+) has the
    symbol A0 L of the comparison medium exactly, A0 drops out of the fixed
    point, and the diffusive part of the operator conserves mass exactly.
    The advective term B . (grad_c chi + g) keeps the central gradient in both.
    Returns chi, grad chi, per-step iteration counts and the status.
    """
    if form not in ("central", "flux"):
        raise ValueError("form must be 'central' or 'flux'")
    if form == "flux" and derivative != "central":
        raise ValueError("the flux form is built on difference operators (derivative='central')")
    H = np.asarray(H)
    shape = H.shape
    d = len(shape)
    Ntot = H.size
    Hf = H.astype(np.float64)
    s, L = symbols(shape, derivative)
    u = np.asarray(u, dtype=np.float64)
    gvec = np.array([float(g[c]) for c in range(d)])
    B0 = np.zeros(d) if B0 is None else np.array([float(B0[c]) for c in range(d)])
    A = diffusivity * (1.0 - Hf) + eta * Hf
    Bf = Pe * (1.0 - Hf) * u
    ubar = pore_mean_velocity(H, u)
    calF = Pe * (1.0 - Hf) * float(ubar @ gvec)
    steady = not math.isfinite(dt)
    inv_dt = 0.0 if steady else 1.0 / dt
    denom = A0 * L + 1j * sum(B0[c] * s[c] for c in range(d)) + inv_dt
    denom = np.broadcast_to(denom, shape).copy()
    if steady:
        denom.flat[0] = 1.0  # k = 0 handled separately below
    B0g_hat = _fft(float(B0 @ gvec) * np.ones(shape))

    chi = np.zeros(shape) if chi_init is None else np.asarray(chi_init, dtype=np.float64).copy()
    chi_hat = _fft(chi)
    grad = grad_spectral(chi_hat, s)
    sqn1 = math.sqrt(Ntot)
    sqn2 = math.sqrt(d * Ntot)
    iters = []
    status = "converged"
    hist = []
    for step in range(n_steps):
        chi_m_hat = chi_hat.copy()
        st = "not_converged"
        it = 0
        r1_min = math.inf
        for it in range(1, max_iter + 1):
            # Step 1: residual F^n in real space
            e = grad + gvec.reshape((d,) + (1,) * d)
            if form == "flux":
                div_tau = sum(backward_diff((face_harmonic_mean(A, c) - A0)
                                            * (forward_diff(chi, c) + gvec[c]), c) for c in range(d))
            else:
                tau_f = (A - A0) * e
                div_tau = _ifft(div_spectral_hat(np.stack([_fft(tau_f[c]) for c in range(d)]), s))
            F = calF + div_tau - sum((Bf[c] - B0[c]) * e[c] for c in range(d))
            # Step 2: solve eq. iter in Fourier (eq. fft_solute)
            num = _fft(F) - B0g_hat + inv_dt * chi_m_hat
            chi_hat_new = num / denom
            if steady:
                chi_hat_new.flat[0] = 0.0
            chi_new = _ifft(chi_hat_new)
            grad_new = grad_spectral(chi_hat_new, s)
            # Step 3: convergence (eq. tol_solute)
            r1 = np.linalg.norm(chi_new - chi)
            r2 = np.linalg.norm(grad_new - grad)
            chi, chi_hat, grad = chi_new, chi_hat_new, grad_new
            if history:
                hist.append((r1, r2))
            # divergence (the LS iteration contracts only for a large enough
            # comparison medium): non-finite, or r_1 grown a millionfold over
            # its smallest value within this time step
            r1_min = min(r1_min, r1)
            if not (np.isfinite(r1) and np.isfinite(r2)) or (it > 5 and r1 > 1e6 * r1_min):
                st = "diverged"
                break
            if r1 <= sqn1 * eps and r2 <= sqn2 * eps:
                st = "converged"
                break
        iters.append(it)
        if st != "converged":
            status = st
            if st == "diverged":
                break
    return dict(chi=chi, grad=grad, iters=iters, status=status, ubar=ubar, history=hist)


# ---------------------------------------------------------------------------
# Effective properties (Section 2, eq. K and eq. D)
# ---------------------------------------------------------------------------

def permeability_darcy(us, nu=1.0):
    """K_ij = (1/nu) h^d sum_Y u^i_j.  At a converged Stokes solution this
    equals the integral of grad u^i . grad u^j (eq. K) because u vanishes in
    the solid and is discretely divergence free."""
    us = [np.asarray(u, dtype=np.float64) for u in us]
    d = us[0].shape[0]
    Ntot = us[0][0].size
    K = np.zeros((len(us), d))
    for i, u in enumerate(us):
        for j in range(d):
            K[i, j] = u[j].sum() / (Ntot * nu)
    return K


def permeability_energy(us):
    """K_ij = h^d sum over voxels and edges of D+u^i . D+u^j (eq. K written
    with forward differences: <u^i, -Delta_h u^j> h^d)."""
    us = [np.asarray(u, dtype=np.float64) for u in us]
    d = us[0].shape[0]
    Ntot = us[0][0].size
    K = np.zeros((len(us), len(us)))
    for i in range(len(us)):
        for j in range(len(us)):
            K[i, j] = sum((us[i][c] * compact_neg_laplacian(us[j][c])).sum() for c in range(d)) / Ntot
    return K


def effective_diffusivity(H, u, chis, Pe):
    """D*_ij = porosity delta_ij + Pe h^d sum_pore (ubar_i - u_i) chi^j
    + h^d sum_pore (grad_c chi^j)_i  (eq. D, component-wise reading of the
    velocity term; central-difference gradient; not divided by porosity)."""
    H = np.asarray(H)
    pore = 1.0 - H.astype(np.float64)
    d = H.ndim
    Ntot = H.size
    por = pore.sum() / Ntot
    ubar = pore_mean_velocity(H, u)
    D = np.zeros((d, len(chis)))
    for j, chi in enumerate(chis):
        gc = central_grad(np.asarray(chi, dtype=np.float64))
        for i in range(d):
            D[i, j] = (por * (1.0 if i == j else 0.0)
                       + Pe * (pore * (ubar[i] - u[i]) * chi).sum() / Ntot
                       + (pore * gc[i]).sum() / Ntot)
    return D


def solute_mass(chi):
    """h^d sum_Y chi."""
    chi = np.asarray(chi, dtype=np.float64)
    return chi.sum() / chi.size


# ---------------------------------------------------------------------------
# Brute-force sparse direct solves of the same discrete equations
# ---------------------------------------------------------------------------

def _shift_matrix(shape, c, k):
    """Sparse permutation P with (P f)(x) = f(x + k h e_c), periodic."""
    nd = len(shape)
    ax = nd - 1 - c
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    src = np.roll(idx, -k, axis=ax).ravel()
    n = idx.size
    return sp.csr_matrix((np.ones(n), (np.arange(n), src)), shape=(n, n))


def _stencil_ops(shape):
    n = int(np.prod(shape))
    nd = len(shape)
    I = sp.identity(n, format="csr")
    G = []
    Lap = sp.csr_matrix((n, n))
    for c in range(nd):
        N = shape[nd - 1 - c]
        Pp = _shift_matrix(shape, c, 1)
        Pm = _shift_matrix(shape, c, -1)
        G.append((Pp - Pm) * (N / 2.0))
        Lap = Lap + (2.0 * I - Pp - Pm) * (N * N)
    return G, Lap  # central gradient components, compact -Delta_h


def brute_force_stokes(H, g, nu=1.0):
    """Discrete constrained Stokes KKT point by a sparse direct solve.

    minimise nu/2 <u, -Delta_h u> - <u, g> over grid velocities with u = 0 on
    solid voxels and central divergence zero at every voxel (the discrete
    form of the constrained variational principle of Section 3.1).  The
    pressure block carries a -delta I regularisation (delta = 1e-13 |A|) so
    that its null modes take their minimum-norm value.
    Returns (u, q) with u of shape (d, *grid).
    """
    H = np.asarray(H)
    shape = H.shape
    nd = len(shape)
    n = H.size
    G, Lap = _stencil_ops(shape)
    fluid = np.flatnonzero(H.ravel() == 0)
    nf = fluid.size
    Lff = (nu * Lap)[fluid][:, fluid]
    blocks_A = sp.block_diag([Lff] * nd, format="csr")
    Gf = sp.vstack([G[c][fluid] for c in range(nd)], format="csr")  # (nd*nf, n)
    scale = abs(blocks_A).max()
    delta = 1e-13 * scale
    K = sp.bmat([[blocks_A, Gf], [Gf.T, -delta * sp.identity(n)]], format="csc")
    rhs = np.concatenate([np.full(nf, float(g[c])) for c in range(nd)] + [np.zeros(n)])
    sol = spla.spsolve(K, rhs)
    u = np.zeros((nd, n))
    for c in range(nd):
        u[c, fluid] = sol[c * nf:(c + 1) * nf]
    q = sol[nd * nf:]
    return u.reshape((nd,) + shape), q.reshape(shape)


def brute_force_transport(H, u, g, Pe, A0=0.55, eta=0.01, diffusivity=1.0,
                          dt=math.inf, chi_prev=None, form="central"):
    """Fixed point of the LS iteration as one sparse linear system.

    Substituting the symbols of eq. fft_app into eq. iter gives, in real space,
      A0 (-Delta_h - div_c grad_c) chi - div_c(A (grad_c chi + g))
        + B . (grad_c chi + g) [+ (chi - chi_prev)/dt] = calF,
    independent of B0 (form="central").  form="flux":
      - sum_c D-_c (A_f,c (D+_c chi + g_c)) + B . (grad_c chi + g)
        [+ (chi - chi_prev)/dt] = calF,
    with forward and backward difference matrices and the face harmonic
    means, independent of A0 and B0.  Steady: bordered with the mean-zero
    constraint.
    """
    H = np.asarray(H)
    shape = H.shape
    nd = len(shape)
    n = H.size
    Hf = H.astype(np.float64).ravel()
    G, Lap = _stencil_ops(shape)
    A = diffusivity * (1.0 - Hf) + eta * Hf
    u = np.asarray(u, dtype=np.float64)
    Bf = [Pe * (1.0 - Hf) * u[c].ravel() for c in range(nd)]
    ubar = pore_mean_velocity(H, u)
    calF = Pe * (1.0 - Hf) * float(sum(ubar[c] * g[c] for c in range(nd)))
    rhs = calF.copy()
    if form == "flux":
        Op = sp.csr_matrix((n, n))
        for c in range(nd):
            N = shape[nd - 1 - c]
            Ieye = sp.identity(n, format="csr")
            Dp = (_shift_matrix(shape, c, 1) - Ieye) * N
            Dm = (Ieye - _shift_matrix(shape, c, -1)) * N
            Af = face_harmonic_mean(A.reshape(shape), c).ravel()
            Op = Op - Dm @ (sp.diags(Af) @ Dp) + sp.diags(Bf[c]) @ G[c]
            rhs = rhs + Dm @ (Af * float(g[c])) - Bf[c] * float(g[c])
    else:
        DivGrad = sum(G[c] @ G[c] for c in range(nd))
        Op = A0 * (Lap + DivGrad)
        Adiag = sp.diags(A)
        for c in range(nd):
            Op = Op - G[c] @ (Adiag @ G[c]) + sp.diags(Bf[c]) @ G[c]
            rhs = rhs + G[c] @ (A * float(g[c])) - Bf[c] * float(g[c])
    if math.isfinite(dt):
        Op = Op + sp.identity(n) / dt
        cp = np.zeros(n) if chi_prev is None else np.asarray(chi_prev, dtype=np.float64).ravel()
        rhs = rhs + cp / dt
        chi = spla.spsolve(Op.tocsc(), rhs)
        return chi.reshape(shape)
    ones = np.ones((n, 1))
    K = sp.bmat([[Op, sp.csr_matrix(ones)], [sp.csr_matrix(ones.T), None]], format="csc")
    sol = spla.spsolve(K, np.concatenate([rhs, [0.0]]))
    return sol[:n].reshape(shape)


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def poiseuille_profile(n_rows, solid_rows, g=1.0, nu=1.0):
    """Exact discrete plane-Poiseuille profile between solid slabs.

    Solid occupies rows [0, solid_rows) along the cross-flow axis of an
    n_rows-periodic grid.  On fluid rows the compact 3-point second
    difference is exact on quadratics, so the discrete solution is
    u(y_j) = g/(2 nu) (y_j - y_a)(y_b - y_j), with y_a, y_b the centres of
    the bounding solid rows.  Returns u over all rows (zero in the solid).
    """
    h = 1.0 / n_rows
    y = (np.arange(n_rows) + 0.5) * h
    ya = (solid_rows - 1 + 0.5) * h
    yb = (n_rows + 0.5) * h
    u = g / (2.0 * nu) * (y - ya) * (yb - y)
    u[:solid_rows] = 0.0
    return u


def diffusion_mode_amplitude(shape, mode, dt, n_steps, A0, form="central"):
    """Amplitude after n backward-Euler steps of a single cosine mode with
    H = 0, Pe = 0: (1 + dt lambda)^(-n), lambda = (1-A0)|s|^2 + A0 L under
    the central/compact symbols of eq. fft_app, or lambda = L in the flux
    form (-D- D+ has the symbol L)."""
    nd = len(shape)
    s2 = 0.0
    Lm = 0.0
    for c in range(nd):
        N = shape[nd - 1 - c]
        th = 2.0 * np.pi * mode[c] / N
        s2 += (np.sin(th) * N) ** 2
        Lm += 4.0 * np.sin(th / 2.0) ** 2 * N * N
    lam = Lm if form == "flux" else (1.0 - A0) * s2 + A0 * Lm
    return (1.0 + dt * lam) ** (-n_steps)
