"""The C-ABI library loads and exports every entry point that include/certglm.h declares (no
compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2502_09502_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "certglm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    decl = declared_functions()
    assert set(decl) == set(_lib.EXPORTS), set(decl) ^ set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_version_status_strings_and_node_defaults():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    lib = _lib.load()
    assert lib.cgl_version() == 1
    assert lib.cgl_status_str(0) == b"ok"
    assert lib.cgl_status_str(1) == b"invalid argument"
    n = _lib.CglNode()
    lib.cgl_node_init(ctypes.byref(n))
    assert n.tol == 1e-6 and n.max_iter == 100000 and n.check_every == 1
    assert n.precision == 0 and n.n_zero == 0 and n.n_in == 0 and n.incumbent == float("inf")


def test_struct_layouts_match_header():
    # cgl_node: two (ptr, int32) pairs, double, 3 int32 + 1 int32, ptr, double
    assert ctypes.sizeof(_lib.CglNode) == 72
    assert ctypes.sizeof(_lib.CglResult) == 56
