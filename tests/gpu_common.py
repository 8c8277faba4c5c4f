"""Helpers for GPU tests: skip cleanly when no GPU, never fall back."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_15554_amd import abi
    abi.load()  # raises if libacm.so is missing: no CPU fallback


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()
