"""The allocation-free effective-properties entry point against the ordinary
one (Section 2, eq. K and eq. D): same fields, the same bits, over two calls
in a row on one GPU, the second with a smaller grid and fewer fields, and in
both precisions and dimensions.  Also checked against the FP64 oracle on the
same fields."""
import numpy as np
import pytest
import torch

from oracle import acm_oracle as O
from paper_2312_15554_amd import inputs as I
from tests.gpu_common import dev, require_gpu


def _fields(shape, seed, n_flow, n_chi):
    d = len(shape)
    H = I.random_mask(shape, seed, 0.35)
    us = [I.random_field((d,) + shape, seed + 10 + k) * (1 - H) for k in range(n_flow)]
    chis = [I.random_field(shape, seed + 20 + k) for k in range(n_chi)]
    return H, us, chis


def _both(H, us, chis, dtype, nu, Pe, stream=None):
    from paper_2312_15554_amd.api import acm_effective_props, acm_effective_props_noalloc
    Hd = dev(H)
    ud = [dev(x, dtype) for x in us]
    cd = [dev(x, dtype) for x in chis]
    ut = ud[0] if chis else None
    ref = acm_effective_props(Hd, ud, cd, u_transport=ut, nu=nu, Pe=Pe)
    got = acm_effective_props_noalloc(Hd, ud, cd, u_transport=ut, nu=nu, Pe=Pe, stream=stream)
    return ref, got


def _same(ref, got):
    for k in ("K", "D", "mass"):
        if ref[k] is None:
            assert got[k] is None
        else:
            assert np.array_equal(ref[k], got[k]), (k, ref[k], got[k])


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_props_equal_props_over_two_calls(dtype):
    """First call 64 x 48 x 32 with three flows and three chi fields, second
    call 16 x 24 x 32 with two flows and one chi field: both bit-equal to
    acm_effective_props, and the second also to the oracle."""
    require_gpu()
    print(f"noalloc props, two calls, dtype={dtype}", flush=True)
    H, us, chis = _fields((32, 48, 64), 3, 3, 3)
    ref, got = _both(H, us, chis, dtype, 0.7, 3.0)
    _same(ref, got)
    H2, us2, chis2 = _fields((16, 24, 32), 5, 2, 1)
    ref2, got2 = _both(H2, us2, chis2, dtype, 1.3, 10.0)
    _same(ref2, got2)
    cast = (lambda a: a.astype(np.float32).astype(np.float64)) if dtype == torch.float32 else (lambda a: a)
    Ko = O.permeability_darcy([cast(x) for x in us2], nu=1.3)
    Do = O.effective_diffusivity(H2, cast(us2[0]), [cast(c) for c in chis2], 10.0)
    assert np.allclose(got2["K"], Ko, rtol=1e-12, atol=1e-14)
    assert np.allclose(got2["D"], Do, rtol=1e-12, atol=1e-13)


@pytest.mark.gpu
def test_noalloc_props_2d_and_k_only_on_a_side_stream():
    """A 2D cell and a K-only call (no chi) on a non-default stream, then a
    smaller 2D cell with D and mass only."""
    require_gpu()
    print("noalloc props, 2D, side stream", flush=True)
    side = torch.cuda.Stream()
    H, us, _ = _fields((64, 96), 7, 2, 0)
    with torch.cuda.stream(side):
        ref, got = _both(H, us, [], torch.float32, 1.0, 0.0, stream=side)
    _same(ref, got)
    H2, us2, chis2 = _fields((16, 32), 8, 1, 2)
    from paper_2312_15554_amd.api import acm_effective_props, acm_effective_props_noalloc
    Hd, ut = dev(H2), dev(us2[0], torch.float32)
    cd = [dev(c, torch.float32) for c in chis2]
    ref2 = acm_effective_props(Hd, [], cd, u_transport=ut, Pe=2.0)
    got2 = acm_effective_props_noalloc(Hd, [], cd, u_transport=ut, Pe=2.0)
    _same(ref2, got2)


@pytest.mark.gpu
def test_noalloc_props_rejects_counts_beyond_its_limit():
    """More than 16 flows is refused before any launch, with a message."""
    require_gpu()
    from paper_2312_15554_amd import abi
    from paper_2312_15554_amd.api import acm_effective_props_noalloc
    H = dev(np.zeros((16, 16, 16), np.uint8))
    u = torch.zeros((3, 16, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(abi.AcmError) as e:
        acm_effective_props_noalloc(H, [u] * 17)
    assert e.value.status == abi.ACM_E_INVALID
    assert "16" in str(e.value)
