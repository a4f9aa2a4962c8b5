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


def _prototypes():
    """name -> [parameter declarations] of every function include/fwime.h declares."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(fwime_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
        params = [p.strip() for p in m.group(2).replace("\n", " ").split(",")]
        out[m.group(1)] = [] if params == ["void"] or params == [""] else params
    return out


def _c_kind(param: str):
    if "*" in param or param.startswith("fwime_objective_fn"):
        return ("ptr", ctypes.sizeof(ctypes.c_void_p))
    base = param.rsplit(" ", 1)[0].replace("const ", "").strip()
    sizes = {"double": ("float", 8), "int32_t": ("int", 4), "int": ("int", 4), "int64_t": ("int", 8),
             "size_t": ("int", ctypes.sizeof(ctypes.c_size_t))}
    return sizes[base]


def _py_kind(t):
    if t in (ctypes.c_double, ctypes.c_float):
        return ("float", ctypes.sizeof(t))
    if t in (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint32):
        return ("int", ctypes.sizeof(t))
    return ("ptr", ctypes.sizeof(ctypes.c_void_p))      # c_void_p, POINTER(...), c_char_p, CFUNCTYPE


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfwime.so not built")
def test_binding_argtypes_match_header_prototypes():
    # a parameter count or kind that differs between the header and the ctypes
    # binding would hand the library misplaced arguments
    from paper_2206_02362_amd import _abi
    lib = _abi.load()
    protos = _prototypes()
    assert sorted(protos) == declared_functions()
    for name, params in protos.items():
        fn = getattr(lib, name)
        assert fn.argtypes is not None, name
        assert len(fn.argtypes) == len(params), (name, len(fn.argtypes), params)
        for p, t in zip(params, fn.argtypes):
            assert _c_kind(p) == _py_kind(t), (name, p, t)
