"""The C-ABI library loads and exports every entry point include/bgktgs.h declares.

CPU-only: loads the shared library with ctypes (no GPU call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2608_19150_amd", "libbgktgs.so")
HDR = os.path.join(ROOT, "include", "bgktgs.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("build_mesh_dag", "tgs_sweep", "moments", "maxwellian", "bgk_step"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_last_error_is_callable_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.bgk_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.bgk_last_error(), bytes)
