"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/fwime.h declares (no compute calls: no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fwime.h")
LIB = os.path.join(ROOT, "paper_2206_02362_amd", "libfwime.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fwime_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_operators():
    names = declared_functions()
    for n in ("fwime_model", "fwime_born_ext_fwd", "fwime_born_ext_adj", "fwime_gradient",
              "fwime_ctx_create", "fwime_ctx_destroy", "fwime_strerror", "fwime_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwime.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwime.so not built")
def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.fwime_strerror.restype = ctypes.c_char_p
    assert lib.fwime_strerror(0) == b"ok"
    assert b"invalid" in lib.fwime_strerror(1)
    assert lib.fwime_strerror(99) == b"unknown error"


def test_python_binding_exports_match_header():
    import paper_2206_02362_amd as fw
    assert sorted(fw.EXPORTED) == declared_functions()
