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


def _c_layout(tmp_path):
    """sizeof / offsetof of the header's structs, from a C program compiled against include/gcharm.h."""
    import subprocess
    fields = {"gc_force_params": [f for f, _ in gc.ForceParams._fields_],
              "gc_ewald_params": [f for f, _ in gc.EwaldParams._fields_],
              "gc_task": list(gc.TASK_DTYPE.names)}
    body = []
    for st, fs in fields.items():
        body.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            body.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "gcharm.h"\nint main(void) {\n' +
                   "\n".join(body) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True)
    return {k: int(v) for k, v in (ln.split() for ln in out.splitlines())}


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's ctypes / numpy records must have the C compiler's sizes and offsets
    lay = _c_layout(tmp_path)
    assert lay["gc_task"] == gc.TASK_DTYPE.itemsize == 40
    for name in gc.TASK_DTYPE.names:
        assert lay[f"gc_task.{name}"] == gc.TASK_DTYPE.fields[name][1], name
    for st, cls in (("gc_force_params", gc.ForceParams), ("gc_ewald_params", gc.EwaldParams)):
        assert lay[st] == ctypes.sizeof(cls), st
        for f, _ in cls._fields_:
            assert lay[f"{st}.{f}"] == getattr(cls, f).offset, (st, f)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(gc, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(gc, "_lib", None)
    with pytest.raises(gc.GcError):
        gc.lib()
