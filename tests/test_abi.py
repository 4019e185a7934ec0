"""The C-ABI library loads and exports what include/hc.h declares (CPU only:
no compute call is made, only host-side argument checking)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(hc_\w+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2412_11809_amd as hc
    if not os.path.exists(hc.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return hc.load_library()


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("hc_cluster", "hc_workspace_size", "hc_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_workspace_size(lib):
    import paper_2412_11809_amd as hc
    assert "gfx950" in hc.hc_version()
    a = hc.hc_workspace_size(1000)
    b = hc.hc_workspace_size(100000)
    assert 0 < a < b
    assert hc.hc_workspace_size(10**6, 448, 512, 16384) > 0


def test_argument_errors_are_synchronous(lib):
    import paper_2412_11809_amd as hc
    k = ctypes.c_int32()
    # n < 0 and a NULL count pointer are rejected before any device work
    assert lib.hc_cluster(None, -1, 10, None, None, ctypes.addressof(k), None) == hc.HC_ERR_ARG
    assert lib.hc_cluster(None, 5, 10, None, None, None, None) == hc.HC_ERR_ARG
    assert lib.hc_cluster(None, 5, 10, None, None, ctypes.addressof(k), None) == hc.HC_ERR_ARG
    assert "NULL" in hc.hc_last_error()
    o = hc._Opts()
    o.width, o.height = 70000, 10
    assert lib.hc_cluster(None, 5, 10, None, None, ctypes.addressof(k), ctypes.byref(o)) == hc.HC_ERR_ARG
