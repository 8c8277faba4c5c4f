"""FP64 CPU oracle of the Fourier-neural-operator warm start.

TEST INFRASTRUCTURE ONLY (tests/, the smoke check and the benchmark's CPU
baseline may use it).  Shares no code with the HIP path.

The network maps the solid indicator H of a periodic cell to an initial guess
(u_x, u_y, u_z, p) for the Stokes ADMM with g = e_x.  It is the standard
Fourier neural operator (Li et al., "Fourier Neural Operator for Parametric
Partial Differential Equations", ICLR 2021), written here from its definition:

    v0 = P_w H + P_b                                   (lift, 1 -> C channels)
    v_{l+1} = act_l( W_l v_l + b_l + K_l v_l ),  l = 0..L-1
        K_l v = irfftn( R_l . rfftn(v) restricted to the kept modes )
        act_l = GELU (tanh form) for l < L-1, identity for the last layer
    h = GELU(Q1 v_L + c1)                              (C -> Cp)
    out = Q2 h + c2                                    (Cp -> 4)

Kept modes: kx in [0, m), ky and kz in [0, m) U [N-m, N) (half spectrum along
x, the last numpy axis).  R_l holds one complex C x C matrix per kept mode.
rfftn is the unnormalised forward transform and irfftn its normalised inverse
(numpy conventions).  All arrays are float64 / complex128.

Shapes: H (B, N, N, N); activations (B, C, N, N, N); R_l (nm, C, C) complex
with modes ordered as returned by kept_modes().
"""
from __future__ import annotations

import math

import numpy as np

GELU_K = math.sqrt(2.0 / math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_K * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    t = np.tanh(GELU_K * (x + 0.044715 * x ** 3))
    dt = (1.0 - t * t) * GELU_K * (1.0 + 3 * 0.044715 * x * x)
    return 0.5 * (1.0 + t) + 0.5 * x * dt


def kept_modes(n, m):
    """Index arrays (kz, ky, kx) of the kept half-spectrum modes, in the
    order kz-major, then ky, then kx."""
    idx = list(range(m)) + list(range(n - m, n))
    kz, ky, kx = np.meshgrid(idx, idx, np.arange(m), indexing="ij")
    return kz.ravel(), ky.ravel(), kx.ravel()


def init_params(C=32, Cp=128, m=12, L=4, seed=0, scale_r=None):
    rng = np.random.Generator(np.random.PCG64(seed))
    nm = (2 * m) * (2 * m) * m
    sr = (1.0 / (C * C)) if scale_r is None else scale_r
    p = dict(C=C, Cp=Cp, m=m, L=L)
    p["Pw"] = rng.standard_normal(C) * 1.0
    p["Pb"] = rng.standard_normal(C) * 0.1
    p["R"] = [sr * (rng.random((nm, C, C)) + 1j * rng.random((nm, C, C))) for _ in range(L)]
    p["W"] = [rng.standard_normal((C, C)) / math.sqrt(C) for _ in range(L)]
    p["b"] = [rng.standard_normal(C) * 0.01 for _ in range(L)]
    p["Q1"] = rng.standard_normal((Cp, C)) / math.sqrt(C)
    p["c1"] = rng.standard_normal(Cp) * 0.01
    p["Q2"] = rng.standard_normal((4, Cp)) / math.sqrt(Cp)
    p["c2"] = np.zeros(4)
    return p


def _spectral(v, R, modes, n):
    """K v for activations v (B, C, n, n, n)."""
    kz, ky, kx = modes
    X = np.fft.rfftn(v, axes=(2, 3, 4))
    Xm = X[:, :, kz, ky, kx]                           # (B, C, nm)
    Ym = np.einsum("moi,bim->bom", R, Xm)
    Y = np.zeros_like(X)
    Y[:, :, kz, ky, kx] = Ym
    return np.fft.irfftn(Y, s=(n, n, n), axes=(2, 3, 4)), Xm


def forward(p, H, keep=False):
    """Network output (B, 4, n, n, n); with keep=True also the cache needed
    by backward()."""
    H = np.asarray(H, dtype=np.float64)
    B, n = H.shape[0], H.shape[-1]
    modes = kept_modes(n, p["m"])
    v = p["Pw"][None, :, None, None, None] * H[:, None] + p["Pb"][None, :, None, None, None]
    cache = dict(H=H, modes=modes, vs=[v], pre=[], Xm=[])
    for l in range(p["L"]):
        k, Xm = _spectral(v, p["R"][l], modes, n)
        pre = np.einsum("oi,bixyz->boxyz", p["W"][l], v) + p["b"][l][None, :, None, None, None] + k
        v = gelu(pre) if l < p["L"] - 1 else pre
        cache["pre"].append(pre)
        cache["Xm"].append(Xm)
        cache["vs"].append(v)
    hp = np.einsum("oi,bixyz->boxyz", p["Q1"], v) + p["c1"][None, :, None, None, None]
    h = gelu(hp)
    out = np.einsum("oi,bixyz->boxyz", p["Q2"], h) + p["c2"][None, :, None, None, None]
    cache["hp"] = hp
    cache["h"] = h
    return (out, cache) if keep else out


def backward(p, cache, dout):
    """Gradients of sum(dout * out) with respect to every parameter.  Complex
    parameters get d/dRe + i d/dIm."""
    n = cache["H"].shape[-1]
    N = n ** 3
    kz, ky, kx = cache["modes"]
    w = np.where((kx == 0) | (2 * kx == n), 1.0, 2.0)    # half-spectrum multiplicity
    g = {}
    h, hp = cache["h"], cache["hp"]
    g["Q2"] = np.einsum("boxyz,bixyz->oi", dout, h)
    g["c2"] = dout.sum(axis=(0, 2, 3, 4))
    dh = np.einsum("oi,boxyz->bixyz", p["Q2"], dout) * gelu_grad(hp)
    v = cache["vs"][-1]
    g["Q1"] = np.einsum("boxyz,bixyz->oi", dh, v)
    g["c1"] = dh.sum(axis=(0, 2, 3, 4))
    dv = np.einsum("oi,boxyz->bixyz", p["Q1"], dh)
    g["R"] = [None] * p["L"]
    g["W"] = [None] * p["L"]
    g["b"] = [None] * p["L"]
    for l in reversed(range(p["L"])):
        pre = cache["pre"][l]
        dpre = dv * gelu_grad(pre) if l < p["L"] - 1 else dv
        vin = cache["vs"][l]
        g["W"][l] = np.einsum("boxyz,bixyz->oi", dpre, vin)
        g["b"][l] = dpre.sum(axis=(0, 2, 3, 4))
        # spectral path: k = irfftn(Y), Y = R X on kept modes, X = rfftn(vin)
        G = np.fft.rfftn(dpre, axes=(2, 3, 4))[:, :, kz, ky, kx] * (w / N)   # dL/dY
        g["R"][l] = np.einsum("bom,bim->moi", G, np.conj(cache["Xm"][l]))
        GX = np.einsum("moi,bom->bim", np.conj(p["R"][l]), G)             # dL/dX
        Z = np.zeros(dpre.shape[:2] + (n, n, n // 2 + 1), dtype=complex)
        Z[:, :, kz, ky, kx] = GX / w
        dv_spec = np.fft.irfftn(Z, s=(n, n, n), axes=(2, 3, 4)) * N
        dv = np.einsum("oi,boxyz->bixyz", p["W"][l], dpre) + dv_spec
    g["Pw"] = np.einsum("bcxyz,bxyz->c", dv, cache["H"])
    g["Pb"] = dv.sum(axis=(0, 2, 3, 4))
    return g


def flat_params(p):
    """List of (name, array) for every trainable parameter."""
    out = [("Pw", p["Pw"]), ("Pb", p["Pb"])]
    for l in range(p["L"]):
        out += [(f"R{l}", p["R"][l]), (f"W{l}", p["W"][l]), (f"b{l}", p["b"][l])]
    out += [("Q1", p["Q1"]), ("c1", p["c1"]), ("Q2", p["Q2"]), ("c2", p["c2"])]
    return out


def grad_of(g, name):
    if name[0] in "RWb" and name[1:].isdigit():
        return g[name[0]][int(name[1:])]
    return g[name]
