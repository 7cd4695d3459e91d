"""The C-ABI library builds, loads and exports every function that
include/ibm.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_09799_amd", "libibm.so")
HEADER = os.path.join(ROOT, "include", "ibm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", text, re.M)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("ibm_tag", "ibm_force", "ibm_viscous", "poisson_solve", "ibm_step",
              "ibm_create", "ibm_destroy", "ibm_check"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libibm.so not built")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    if not os.path.exists(LIB):
        pytest.skip("libibm.so not built")
    from paper_2606_09799_amd import ibm
    assert set(_declared()) <= set(ibm.EXPORTS)


def test_strerror_is_callable_without_a_device():
    if not os.path.exists(LIB):
        pytest.skip("libibm.so not built")
    lib = ctypes.CDLL(LIB)
    lib.ibm_strerror.restype = ctypes.c_char_p
    assert lib.ibm_strerror(-1)
    assert b"capacity" in lib.ibm_strerror(-4)
