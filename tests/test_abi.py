"""The C ABI library loads and exports every function declared in include/*.h
(no GPU needed; no compute call is made)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2009_01967_amd", "libkaldo.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"\b(kaldo_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for required in ["kaldo_phonons", "kaldo_linewidths", "kaldo_kappa_rta", "kaldo_kappa_qhgk",
                     "kaldo_create", "kaldo_destroy", "kaldo_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkaldo.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkaldo.so not built")
def test_binding_names_match_header():
    from paper_2009_01967_amd import kaldo
    for n in declared_functions():
        assert hasattr(kaldo, n), n
    assert sorted(kaldo.EXPORTED) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2009_01967_amd import kaldo
    saved = kaldo._lib
    kaldo._lib = None
    try:
        with pytest.raises(ImportError):
            kaldo.load_library(str(tmp_path / "none.so"))
    finally:
        kaldo._lib = saved
