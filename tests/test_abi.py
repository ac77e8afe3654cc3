"""The C-ABI library loads and exports every entry point include/rmb.h
declares (no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmb.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rmb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path_calls():
    syms = declared_symbols()
    for name in ("rmb_ctx_create", "rmb_mobility_matvec"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (one HIP runtime for torch and the library)
    import paper_1602_02170_amd as rmb
    if not os.path.exists(rmb.LIB_PATH):
        pytest.fail("librmb.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(rmb.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(rmb.EXPORTS) == declared_symbols()
    lib.rmb_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.rmb_version()


def test_binding_refuses_to_run_without_library(tmp_path):
    import paper_1602_02170_amd as rmb
    old = rmb._LIB
    rmb._LIB = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            rmb.library(str(tmp_path / "missing.so"))
    finally:
        rmb._LIB = old
