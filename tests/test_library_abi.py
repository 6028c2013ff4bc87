"""The C ABI library loads and exports every function include/lq.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lq_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("lq_create", "lq_destroy", "lq_upload_gauge", "lq_dslash",
                     "lq_clover_apply", "lq_solve"):
        assert required in names


def test_library_exports_all_declared_symbols():
    from paper_1103_1363_amd import lq
    if not os.path.exists(lq.LIB_PATH):
        pytest.fail("liblq.so is not built (run python -m paper_1103_1363_amd.build)")
    lib = ctypes.CDLL(lq.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1103_1363_amd import lq
    monkeypatch.setattr(lq, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lq, "_lib", None)
    with pytest.raises(ImportError):
        lq.lib()
