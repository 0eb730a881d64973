"""The C ABI: the built library loads and exports every function that
include/hgs.h declares, and the Python binding marshals exactly those.  No
call that needs a GPU is made here."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hgs.h")


def declared_functions() -> list[str]:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)  # drop comments
    names = re.findall(r"^\s*(?:hgs_status|void|const char\s*\*)\s*(hgs_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("hgs_create", "hgs_destroy", "hgs_upload", "hgs_cut", "hgs_render", "hgs_render_backward"):
        assert n in names, n


def test_library_exports_every_declared_function():
    from paper_2406_12080_amd import hgs
    if not os.path.exists(hgs.LIB_PATH):
        pytest.fail(f"{hgs.LIB_PATH} is not built (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(hgs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2406_12080_amd import hgs
    assert sorted(hgs.EXPORTS) == declared_functions()


def test_binding_without_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2406_12080_amd import hgs
    monkeypatch.setattr(hgs, "_lib", None)
    monkeypatch.setattr(hgs, "LIB_PATH", str(tmp_path / "libhgs.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        hgs.lib()
