"""The C-ABI library loads and exports every function include/ompd.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2406_13881_amd as ompd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ompd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(ompd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("ompd_analyze_cfg", "ompd_analyze_batch", "ompd_submit", "ompd_poll", "ompd_plan_run"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports(name):
    lib = ompd.lib()
    assert hasattr(lib, name), name
    assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_no_silent_fallback(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of computing."""
    monkeypatch.setattr(ompd, "_SO", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ompd, "_handle", None)
    with pytest.raises(ompd.OmpdNotBuilt):
        ompd.lib()
