"""CPU checks of the C-ABI library: it loads and exports what the header declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "berryhip.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(be_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_five_calls():
    names = declared()
    for n in ("be_build_hk", "be_eigh_batched", "be_wilson_loop", "be_nested_wilson", "be_spin_resolved_wilson"):
        assert n in names


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2312_13051_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    for n in declared():
        assert hasattr(lib, n), n
    assert set(_lib.EXPORTS) == set(declared())
