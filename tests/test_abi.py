"""The C-ABI library loads and exports every entry point include/lrt.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

from paper_2604_11856_amd import lrt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "lrt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lrt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_surface():
    assert set(declared_symbols()) == set(lrt.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(lrt.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing


def test_version_and_status_strings_without_device():
    L = lrt.lib()
    assert L.lrt_version().decode().count(".") == 2
    assert L.lrt_status_string(0).decode() == "ok"
    assert L.lrt_status_string(4).decode() == "over budget"


def test_create_rejects_null_out():
    L = lrt.lib()
    assert L.lrt_create(0, None) == 1
