"""The C-ABI library loads and exports every function include/cm.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "cm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("cm_geometry_create", "cm_collide", "cm_collide_backward", "cm_server_submit",
                     "cm_server_poll"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2602_20304_amd import _lib
    lib = _lib.load()
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(header_functions()) == set(_lib.SIGNATURES)


def test_status_strings_without_device():
    from paper_2602_20304_amd import _lib
    lib = _lib.load()
    assert lib.cm_status_str(0) == b"ok"
    assert lib.cm_status_str(-7) == b"capacity exceeded"
    assert lib.cm_geometry_count(None) == -1
