"""The C-ABI library loads without a GPU and exports every symbol the header
declares (no compute calls here)."""
import ctypes
import os
import re

from paper_1804_04640_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "fastcount.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for want in ("fc_db_create", "fc_count", "fc_count_batch", "fc_count_reduce"):
        assert want in names
    assert sorted(_lib.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name


def test_last_error_is_empty_string_initially():
    assert _lib.load().fc_last_error() == b""


def test_null_handle_is_rejected_without_device_work():
    L = _lib.load()
    assert L.fc_db_info(None, None, None, None, None) == _lib.FC_ERR_INVALID
    assert b"NULL" in L.fc_last_error()
