"""The C-ABI library loads and exports every entry point declared in include/edfa.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "edfa.h")
LIB = os.path.join(ROOT, "paper_2009_13916_amd", "libedfa.so")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:edfa_status|void|const char \*)\s*(edfa_\w+)\s*\(", txt, re.M)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("edfa_assemble", "edfa_setup", "edfa_solve", "edfa_apply", "edfa_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_path_without_gpu_work():
    """A NULL argument is rejected before any device call, with a message."""
    lib = ctypes.CDLL(LIB)
    lib.edfa_assemble.restype = ctypes.c_int
    lib.edfa_last_error.restype = ctypes.c_char_p
    st = lib.edfa_assemble(None, 0, None, None)
    assert st == -1
    assert b"NULL" in lib.edfa_last_error() or b"grid" in lib.edfa_last_error()
