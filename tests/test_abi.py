"""The C ABI library loads (no GPU needed) and exports every function that
include/bks.h declares; the binding's symbol list matches the header."""
import ctypes
import os
import re

import pytest

from paper_2012_07595_amd import bks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "bks.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("bks_", "hooi_"))))


def test_header_lists_entry_points():
    names = header_functions()
    for must in ("bks_tensor_upload", "bks_ttmc", "bks_solve", "hooi_solve"):
        assert must in names
    assert sorted(bks.SYMBOLS) == names


def test_library_exports_every_symbol():
    if not os.path.exists(bks.LIBPATH):
        pytest.skip("libbks.so not built")
    lib = ctypes.CDLL(bks.LIBPATH)
    for name in header_functions():
        assert hasattr(lib, name), name


def test_version_string():
    if not os.path.exists(bks.LIBPATH):
        pytest.skip("libbks.so not built")
    lib = bks.load()
    assert b"gfx950" in lib.bks_version()


def test_ctx_create_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available() or not os.path.exists(bks.LIBPATH):
        pytest.skip("GPU present or library not built")
    lib = bks.load()
    h = ctypes.c_void_p()
    rc = lib.bks_ctx_create(0, 0, ctypes.byref(h))
    assert rc == bks.EDEVICE
