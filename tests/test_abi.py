"""The C-ABI library loads and exports every symbol include/mcx.h declares
(CPU-only: no compute calls)."""
import ctypes
import os
import re

import pytest

import paper_2003_00796_amd as mcx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "mcx.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char\*) (mcx_[a-z_]+)\(", src, re.M)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(mcx.ABI_SYMBOLS)


@pytest.mark.skipif(not os.path.exists(mcx.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(mcx.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(mcx.LIB_PATH), reason="library not built")
def test_create_rejects_bad_arguments_without_touching_a_kernel():
    L = mcx.lib()
    h = ctypes.c_void_p()
    assert L.mcx_create(ctypes.byref(h), 0, 7) == -1  # bad precision
    assert L.mcx_create(None, 0, 0) == -1
    assert L.mcx_last_error(None) == b"null context"
