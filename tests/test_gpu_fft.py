"""Multi-dimensional R2C/C2R transforms of the HIP path against numpy."""
import numpy as np
import pytest
import torch

from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, host, require_gpu

SHAPES = [(8, 8), (16, 24), (64, 64), (48, 96), (8, 16, 24), (16, 16, 16), (32, 48, 64),
          (24, 32, 16), (128, 128, 128),
          # 256- and 512-long axes along x (rows), y and z (columns)
          (8, 16, 256), (256, 8, 16), (16, 256, 8), (256, 256), (8, 8, 512), (512, 8, 8),
          (192, 16, 16)]


@pytest.mark.gpu
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_r2c_matches_numpy_and_roundtrips(shape, dtype):
    require_gpu()
    from paper_2312_15554_amd.api import acm_fft_c2r, acm_fft_r2c
    print(f"fft shape={shape} dtype={dtype}", flush=True)
    x = I.random_field((2,) + shape, seed=sum(shape))
    X = acm_fft_r2c(dev(x, dtype), shape)
    torch.cuda.synchronize()
    ref = np.stack([np.fft.rfftn(x[k]) for k in range(2)])
    err = np.abs(host(X) - ref).max() / np.abs(ref).max()
    tol = 1e-13 if dtype == torch.float64 else 3e-6
    assert err < tol, err
    y = acm_fft_c2r(X, shape)
    err2 = np.abs(host(y) - x).max() / np.abs(x).max()
    assert err2 < tol, err2
