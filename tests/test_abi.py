"""The C-ABI library loads and exports every function include/tw.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "tw.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tw_[a-z_]+)\s*\(", text)))


def _lib_path():
    import paper_2605_16182_amd as tw
    if not os.path.exists(tw.LIB_PATH):
        from paper_2605_16182_amd import build
        build.build()
    return tw.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for f in ("tw_create", "tw_destroy", "tw_ingest_batch", "tw_evict_before",
              "tw_sample_walks", "tw_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_rejects_calls_without_library(monkeypatch, tmp_path):
    import paper_2605_16182_amd as tw
    monkeypatch.setattr(tw, "_lib", None)
    monkeypatch.setattr(tw, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        tw.lib()


def test_null_arguments_fail_cleanly():
    lib = ctypes.CDLL(_lib_path())
    lib.tw_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.tw_last_error.restype = ctypes.c_char_p
    assert lib.tw_create(None, None) == 1  # TW_EINVAL, no device touched
    assert b"null" in lib.tw_last_error()
