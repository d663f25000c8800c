"""The C-ABI library loads and exports every function include/qtx_rgf.h declares
(no GPU needed: only dlopen + symbol lookup, no compute call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qtx_rgf.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qtx_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("qtx_rgf_create", "qtx_rgf_solve", "qtx_rgf_destroy"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_2606_25595_amd import qtx
    if not os.path.exists(qtx.LIB_PATH):
        pytest.fail("libqtx_rgf.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(qtx.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(qtx.EXPORTED)


def test_status_strings_without_gpu():
    from paper_2606_25595_amd import qtx
    assert qtx.status_str(qtx.QTX_OK) == "QTX_OK"
    assert qtx.status_str(qtx.QTX_ERR_SINGULAR) == "QTX_ERR_SINGULAR"
