"""The C-ABI library loads and exports every entry point include/gcharm.h declares (CPU only, no compute)."""
import ctypes
import os
import re

import pytest

import paper_2008_05712_amd as gc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "gcharm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:gc_status|const char\*)\s+(gc_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_documented_entry_points():
    names = _declared()
    for must in ["gc_pool_create", "gc_pool_place", "gc_submit_tasks", "gc_reorganize", "gc_launch_combined",
                 "gc_backward", "gc_graph_capture", "gc_autotune"]:
        assert must in names
    assert sorted(names) == sorted(gc.EXPORTED)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(gc.LIB_PATH):
        pytest.skip("libgcharm.so not built")
    lib = ctypes.CDLL(gc.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert b"gfx950" in gc.lib().gc_version()


def test_task_record_layout():
    assert gc.TASK_DTYPE.itemsize == 40
    assert ctypes.sizeof(gc.ForceParams) == 4 * 4 + 3 * 8 + 4 * 5 + 4  # with alignment padding


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(gc, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(gc, "_lib", None)
    with pytest.raises(gc.GcError):
        gc.lib()
