"""CPU-only: the C-ABI library loads and exports every symbol include/me.h declares (no
compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2210_11122_amd", "libme.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "me.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b([a-z_]+)\s*\([^;{]*\)\s*;", src)
    return sorted(set(n for n in names if n.startswith(("me_", "rambo_"))))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["me_create", "rambo_momenta", "me_sigma", "me_destroy", "me_info", "me_last_error"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libme.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libme.so not built")
def test_binding_export_list_matches_header():
    from paper_2210_11122_amd import binding
    assert sorted(binding.EXPORTS) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libme.so not built")
def test_host_only_argument_checks():
    """entry points that reject a NULL handle before any device call"""
    lib = ctypes.CDLL(LIB)
    lib.me_set_option.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.me_last_error.restype = ctypes.c_char_p
    assert lib.me_set_option(None, 1, 1) == -1
    assert b"NULL" in lib.me_last_error()
