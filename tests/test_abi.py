"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scabs.h")
LIB = os.path.join(ROOT, "paper_1004_5076_amd", "libscabs.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scabs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("scabs_create", "scabs_set_mesh", "scabs_set_media", "scabs_build", "scabs_matvec",
                     "scabs_solve", "scabs_rhs_dipole", "scabs_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libscabs.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_match_header():
    import paper_1004_5076_amd as pk
    assert sorted(pk.EXPORTED) == declared()


def test_argument_errors_without_gpu():
    """Null arguments are rejected before any device work."""
    lib = ctypes.CDLL(LIB)
    lib.scabs_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.scabs_create(None, None) == -1
    lib.scabs_matvec.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_int]
    assert lib.scabs_matvec(None, None, None, 1, 0) == -1
    lib.scabs_precond_apply.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int] * 3
    assert lib.scabs_precond_apply(None, None, None, 1, 0, 0) == -1
    lib.scabs_profile_mask.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    assert lib.scabs_profile_mask(None, 1) == -1
    lib.scabs_last_error.restype = ctypes.c_char_p
    lib.scabs_last_error.argtypes = [ctypes.c_void_p]
    assert lib.scabs_last_error(None) == b"null context"
