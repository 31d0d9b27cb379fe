"""The C-ABI library loads on the CPU and exports every function that
include/dpba.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dpba.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s+(ba_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("ba_create", "ba_solve", "ba_backward", "ba_status", "ba_last_error", "ba_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2208_04726_amd import native
    if not os.path.exists(native.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(native.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(native.EXPORTED)


def test_structs_match_header_layout():
    from paper_2208_04726_amd import native
    # ba_config: 2 int32, 2 double, 4 int32, 3 int64
    assert ctypes.sizeof(native.BAConfig) == 8 + 16 + 16 + 24
    # ba_problem: 2 int32 + 14 pointers
    assert ctypes.sizeof(native.BAProblem) == 8 + 14 * 8
