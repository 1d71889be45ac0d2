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


STRUCTS = [("bks_params", bks.Params), ("bks_info", bks.Info), ("hooi_params", bks.HooiParams),
           ("bks_gparams", bks.GParams), ("bks_server_params", bks.ServerParams),
           ("bks_result", bks.Result)]


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets (a C program built against include/bks.h prints them): a field
    added on one side only would shift everything after it."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bks.h"', "int main(void) {"]
    for cname, py in STRUCTS:
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            cf = fname.lstrip("_")
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, field, value = line.split()
            got[(cname, field)] = int(value)
    for cname, py in STRUCTS:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
