"""CPU-side checks of the C ABI: the library builds, loads without a GPU and
exports every entry point include/msc.h declares; the binding's signature
table covers exactly those names; the product path has no CPU fallback."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "msc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(msc_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("msc_init", "msc_bdf2_step", "msc_explicit_step", "msc_moments", "msc_free"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2609_39474_amd import msc
    if not os.path.exists(msc.LIB_PATH):
        pytest.skip("libmsc_hip.so not built")
    L = ctypes.CDLL(msc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_the_header():
    from paper_2609_39474_amd import msc
    assert sorted(msc.SIGNATURES) == declared_functions()


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2609_39474_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"(import\s+oracle|from\s+oracle|liboracle|orc_[a-z])", src), fn


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2609_39474_amd import msc
    monkeypatch.setattr(msc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(msc, "_lib", None)
    with pytest.raises(RuntimeError):
        msc.lib()
