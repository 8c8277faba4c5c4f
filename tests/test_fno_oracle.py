"""Pins for the FNO oracle: backward() against central finite differences of
forward() on a tiny network (8^3 cell, 4 channels, 2 modes), and the
spectral-convolution path against a direct DFT sum."""
import numpy as np
import pytest

from oracle import fno_oracle as F
from paper_2312_15554_amd import inputs as I


def _setup():
    p = F.init_params(C=4, Cp=6, m=2, L=2, seed=3, scale_r=0.3)
    H = np.stack([I.random_mask((8, 8, 8), s, 0.4).astype(float) for s in (1, 2)])
    dout = I.random_field((2, 4, 8, 8, 8), 9)
    return p, H, dout


@pytest.mark.parametrize("name", ["Pw", "Pb", "R0", "R1", "W0", "W1", "b0", "b1", "Q1", "c1", "Q2", "c2"])
def test_backward_matches_finite_differences(name):
    p, H, dout = _setup()
    out, cache = F.forward(p, H, keep=True)
    g = F.backward(p, cache, dout)
    arr = dict(F.flat_params(p))[name]
    ga = F.grad_of(g, name)
    rng = np.random.Generator(np.random.PCG64(0))
    flat = arr.reshape(-1)
    gflat = ga.reshape(-1)
    for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
        parts = [(1.0, "re")] + ([(1j, "im")] if np.iscomplexobj(arr) else [])
        for unit, part in parts:
            h = 1e-6
            old = flat[idx]
            flat[idx] = old + h * unit
            lp = (F.forward(p, H) * dout).sum()
            flat[idx] = old - h * unit
            lm = (F.forward(p, H) * dout).sum()
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = gflat[idx].real if part == "re" else gflat[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, part, fd, an)


def test_spectral_path_equals_direct_dft():
    """K v computed by rfftn/irfftn equals the explicit mode sum
    (1/N) sum_k conj-completed Y(k) exp(2 pi i k.x / n) for one channel."""
    n, m = 6, 2
    rng = np.random.Generator(np.random.PCG64(1))
    v = rng.standard_normal((1, 1, n, n, n))
    R = rng.standard_normal((4 * m * m * m // 2 * 2, 1, 1)) + 1j * rng.standard_normal((4 * m * m * m // 2 * 2, 1, 1))
    modes = F.kept_modes(n, m)
    R = R[: len(modes[0])]
    k, _ = F._spectral(v, R, modes, n)
    # direct: X(k) by explicit sum, Y = R X on kept modes, full Hermitian inverse
    x = np.arange(n)
    Z, Y_, X_ = np.meshgrid(x, x, x, indexing="ij")
    full = np.zeros((n, n, n), complex)
    for j, (kz, ky, kx) in enumerate(zip(*modes)):
        ph = np.exp(-2j * np.pi * (kz * Z + ky * Y_ + kx * X_) / n)
        Xk = (v[0, 0] * ph).sum()
        Yk = R[j, 0, 0] * Xk
        full[kz, ky, kx] += Yk
        if 0 < kx < n - kx:  # the conjugate partner of a half-spectrum mode
            full[(-kz) % n, (-ky) % n, (-kx) % n] += np.conj(Yk)
    direct = np.zeros((n, n, n))
    for kz in range(n):
        for ky in range(n):
            for kx in range(n):
                if full[kz, ky, kx] != 0:
                    direct += (full[kz, ky, kx] * np.exp(2j * np.pi * (kz * Z + ky * Y_ + kx * X_) / n)).real
    direct /= n ** 3
    assert np.allclose(k[0, 0], direct, atol=1e-12)
