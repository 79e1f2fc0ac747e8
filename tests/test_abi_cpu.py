"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lineset.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b((?:lineset|ls)_\w+)\s*\(", text,
                       flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("lineset_voxelize", "lineset_build_lod", "lineset_render", "lineset_destroy",
              "lineset_export", "lineset_info", "ls_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1801_01155_amd as L
    lib = L.lib()
    for n in _declared():
        assert hasattr(lib, n), f"{n} not exported"
    out = subprocess.check_output(["nm", "-D", "--defined-only", L.LIB_PATH]).decode()
    exported = set(re.findall(r" T (\w+)$", out, flags=re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_error_text_without_gpu():
    import paper_1801_01155_amd as L
    lib = L.lib()
    assert lib.ls_version() >= 100
    assert isinstance(lib.ls_last_error(), bytes)
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    rc = lib.lineset_voxelize(None, None, ctypes.byref(h))
    assert rc == L.LS_EINVAL and h.value is None
    assert b"desc" in lib.ls_last_error()


def test_product_package_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_1801_01155_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "lineset_oracle" not in src, f
