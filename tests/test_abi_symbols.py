"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "acm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(acm_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["acm_stokes_solve", "acm_transport_step", "acm_effective_props", "acm_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    path = os.path.join(ROOT, "paper_2312_15554_amd", "libacm.so")
    if not os.path.exists(path):
        pytest.skip("libacm.so not built")
    lib = ctypes.CDLL(path)
    for n in _declared():
        assert hasattr(lib, n), n
    from paper_2312_15554_amd import abi
    assert set(abi.SIGNATURES) == set(_declared())
    lib.acm_version.restype = ctypes.c_int32
    assert lib.acm_version() == abi.ABI_VERSION
