"""The C ABI library builds, loads and exports every symbol the header declares
(no compute: these run without a GPU)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "ara.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ara_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("ara_load_yet", "ara_load_elts", "ara_run_layer", "ara_risk_measures",
                 "ara_create", "ara_destroy", "ara_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import paper_1310_2274_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libara.so not built")
    L = ctypes.CDLL(P.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_binding_signatures_cover_the_header():
    import paper_1310_2274_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libara.so not built")
    L = P.lib()
    for s in declared_symbols():
        assert getattr(L, s).argtypes is not None, s
        assert hasattr(P, s), f"binding lacks {s}"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_1310_2274_amd as P
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError):
        P.lib()


def test_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1310_2274_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), f
                assert "ara_oracle" not in src, f
