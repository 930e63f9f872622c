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


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No fallback: without the built library the binding raises."""
    monkeypatch.setattr(khcore, "_lib", None)
    with pytest.raises(ImportError):
        khcore.load_library(str(tmp_path / "absent.so"))


def test_null_arguments_of_newer_entry_points():
    if not os.path.exists(khcore.LIB_PATH):
        pytest.skip("library not built")
    lib = khcore.load_library()
    assert lib.khc_autotune(None, None, 3, 8, None) == khcore.KHC_EINVAL
    assert lib.khc_set_progress(None, khcore.PROGRESS_FN(), None, 100) == khcore.KHC_EINVAL
    assert lib.khc_persist_profile_read(None, None, None, 0) == khcore.KHC_EINVAL
    assert lib.khc_mlp_save(None, None, b"x") == khcore.KHC_EINVAL
    assert lib.khc_mlp_load(None, None, b"x") == khcore.KHC_EINVAL
    assert lib.khcore_decompose_approx(None, None, 3, None, None, None, None) == khcore.KHC_EINVAL
