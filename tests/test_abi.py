"""The C ABI library loads and exports every function include/pmg.h declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:int|const char\s*\*)\s+(\w+)\s*\(", text, flags=re.M)
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pmg_patch_setup", "pmg_patch_smooth", "gmg_cg_solve", "pmg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2510_17785_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpmg.so is not built (python -m paper_2510_17785_amd.build)")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(declared_functions()) == sorted(_lib.EXPORTS)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2510_17785_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError):
        _lib.load()
