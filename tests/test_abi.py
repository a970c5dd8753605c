"""The C ABI: the library loads and exports every entry point include/hgl.h
declares, and the Python binding declares the same set.  No GPU needed."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(hgl_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_boundary():
    names = declared()
    for must in ["hgl_build_laplacian", "hgl_cg_solve", "hgl_apply", "hgl_destroy", "hgl_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1908_08281_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhgl.so is not built (run python -m paper_1908_08281_amd.build)")
    lib = _lib.load()
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    assert lib.hgl_version() >= 100


def test_binding_covers_every_declared_symbol():
    from paper_1908_08281_amd import _lib
    assert declared() == set(_lib.SIGNATURES), (declared() ^ set(_lib.SIGNATURES))


def test_oracle_not_imported_by_product():
    pkg = os.path.join(ROOT, "paper_1908_08281_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, flags=re.M), f
