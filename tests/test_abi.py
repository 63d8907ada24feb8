"""The C-ABI library loads on the CPU and exports every entry point that
include/uvmem.h declares (no compute: there may be no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "uvmem.h")
LIB = os.path.join(ROOT, "paper_1703_02920_amd", "libuvmem.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(uvmem_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared()
    for required in ("uvmem_create", "uvmem_set_uv", "uvmem_set_vis", "uvmem_set_weights", "uvmem_set_beam",
                     "uvmem_set_prior", "uvmem_finalize", "uvmem_phi_and_grad", "uvmem_forward",
                     "uvmem_adjoint", "uvmem_cg_init", "uvmem_cg_step", "uvmem_cg_run"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        from paper_1703_02920_amd import build
        build.build(verbose=False)
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_symbol_list_matches_header():
    from paper_1703_02920_amd import uvmem
    assert sorted(uvmem.SYMBOLS) == declared()


def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.uvmem_strerror.restype = ctypes.c_char_p
    assert lib.uvmem_strerror(0) == b"ok"
    assert lib.uvmem_strerror(-4).startswith(b"image pixel")
    lib.uvmem_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_void_p]
    h = ctypes.c_void_p()
    # odd image side is rejected before any device call
    assert lib.uvmem_create(ctypes.byref(h), 63, 1, 0, 1, None) == -1
    assert lib.uvmem_create(None, 64, 1, 0, 1, None) == -1
