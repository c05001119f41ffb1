"""CPU checks of the C ABI: the built library loads and exports every entry
point include/sps.h declares, and the Python binding names match."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sps.h")
LIB = os.path.join(ROOT, "paper_1304_4333_amd", "libsps.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sps_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("sps_loglik", "sps_loglik_grad", "sps_correct", "sps_resample", "sps_mutate", "sps_logml"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libsps.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"


def test_binding_covers_the_abi():
    from paper_1304_4333_amd import sps
    assert sorted(sps.ABI_NAMES) == _declared()
