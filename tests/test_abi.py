"""Host-side checks of the C ABI: the library loads, exports every declared
entry point, and its pure-host calls behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccgpu.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(cc_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2510_12053_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    return ctypes.CDLL(b.LIB)


def test_header_declares_entry_points():
    names = _declared()
    for must in ("cc_create", "cc_destroy", "cc_mesh_upload", "cc_color", "cc_layout",
                 "cc_subspace_upload", "cc_subspace_build", "cc_step"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_symbol():
    import paper_2510_12053_amd.ccgpu as cg
    src = open(cg.__file__).read()
    missing = [n for n in _declared() if f'"{n}"' not in src]
    assert not missing, missing


def test_params_default(lib):
    import paper_2510_12053_amd.ccgpu as cg
    p = cg.cc_params_default()
    assert (p.method, p.sweep, p.precision, p.line_search, p.max_iters, p.max_halvings,
            p.corotate) == (cg.METHOD_CC, cg.SWEEP_JACOBI, cg.FP64, 1, 10000, 20, 0)
    # the binding's struct has the size of the C struct (the header's field list)
    assert ctypes.sizeof(cg.cc_params) == 4 * 9 + 4 + 8 * 3 + 4 + 4


def test_null_arguments_rejected(lib):
    lib.cc_create.restype = ctypes.c_int32
    lib.cc_create.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.cc_create(0, None, None) == -1          # CC_E_INVALID_ARG
    lib.cc_step.restype = ctypes.c_int32
    assert lib.cc_step(None, 0, None, None, None, ctypes.c_double(0.1), None,
                       ctypes.c_double(1e-6), None, None) == -1
    lib.cc_last_error.restype = ctypes.c_char_p
    assert lib.cc_last_error(None) == b"null context"
