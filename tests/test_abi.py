"""The C-ABI library loads and exports every symbol include/khcore.h declares
(no compute calls: CPU only)."""
import ctypes
import os
import re

import pytest

from paper_2006_03372_amd import khcore

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|const char \*)\s*(\w+)\s*\(", text, re.M))
    return names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(khcore.LIB_PATH):
        pytest.skip("library not built")
    lib = khcore.load_library()
    declared = _declared()
    assert declared, "no declarations found"
    assert set(khcore.EXPORTED) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_null_context_is_rejected_without_gpu():
    if not os.path.exists(khcore.LIB_PATH):
        pytest.skip("library not built")
    lib = khcore.load_library()
    assert lib.khc_set_option(None, 1, 4) == khcore.KHC_EINVAL
    assert lib.khdeg_compute(None, None, None, 2, None) == khcore.KHC_EINVAL
    assert lib.khcore_decompose(None, None, 2, None, None, None) == khcore.KHC_EINVAL
    assert lib.khc_last_error(None) == b"null context"
