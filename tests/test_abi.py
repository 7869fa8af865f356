"""The C-ABI library loads and exports every function include/chfsi.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfsi.h")
LIB = os.path.join(ROOT, "paper_2203_07820_amd", "libchfsi.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["chfsi_op_build", "chfsi_apply", "chfsi_filter", "chfsi_orthonormalize",
              "chfsi_rayleigh_ritz", "chfsi_solve", "chfsi_bounds"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_declares_every_symbol():
    from paper_2203_07820_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    lib = _lib.load()
    assert lib.chfsi_version().decode().startswith("chfsi")


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_struct_layouts_match_the_library():
    from paper_2203_07820_amd import _lib
    lib = _lib.load()
    sizes = [ctypes.c_int64() for _ in range(3)]
    assert lib.chfsi_abi_sizes(*[ctypes.byref(x) for x in sizes]) == 0
    assert [x.value for x in sizes] == [ctypes.sizeof(_lib.System), ctypes.sizeof(_lib.Params),
                                        ctypes.sizeof(_lib.Stats)]
