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
    o.width, o.height, o.flags = 256, 256, hc.HC_FLAG_LINK_PIXEL_INDEX | hc.HC_FLAG_LINK_WINDOW
    assert lib.hc_cluster(None, 0, 10, None, None, ctypes.addressof(k), ctypes.byref(o)) == hc.HC_ERR_ARG
    assert "flags" in hc.hc_last_error()


def test_batch_argument_errors_are_synchronous(lib):
    import numpy as np
    import paper_2412_11809_amd as hc
    lib = hc._bind_batch(lib)
    i64 = ctypes.POINTER(ctypes.c_int64)
    u64 = ctypes.POINTER(ctypes.c_uint64)
    k = ctypes.c_int32()

    def call(offsets, n_chunks, dts):
        o = np.asarray(offsets, dtype=np.int64)
        d = np.asarray(dts, dtype=np.uint64)
        return lib.hc_cluster_batch(None, o.ctypes.data_as(i64), n_chunks, d.ctypes.data_as(u64), None, None,
                                    ctypes.addressof(k), None, None)
    assert call([0], 0, []) == hc.HC_ERR_ARG                      # no chunks
    assert call([1, 5], 1, [10]) == hc.HC_ERR_ARG                 # offsets[0] != 0
    assert call([0, 5, 3], 2, [10, 10]) == hc.HC_ERR_ARG          # decreasing offsets
    assert call([0, 1 << 31], 1, [10]) == hc.HC_ERR_OVERFLOW      # more than 2^31 - 1 hits
    assert call([0, 5], 1, [10]) == hc.HC_ERR_ARG                 # NULL hits/labels
    out = ctypes.c_void_p()
    assert lib.hc_batch_graph_create(None, None, 1, None, None, None, None, None, None,
                                     ctypes.byref(out)) == hc.HC_ERR_ARG
    assert lib.hc_batch_autotune(None, None, 1, None, None, None, None, None, None) == hc.HC_ERR_ARG
    assert lib.hc_batch_graph_launch(None, None) == hc.HC_ERR_ARG
    lib.hc_batch_plan_destroy(None)
    lib.hc_batch_graph_destroy(None)
    a = hc.hc_batch_workspace_size([0, 100, 5000, 5000, 20000])
    b = hc.hc_batch_workspace_size([0, 20000])
    assert a > 0 and b > 0


def test_binding_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof of every struct in hc.h, compiled with gcc, equal the
    ctypes/numpy layouts of the binding."""
    import subprocess
    import numpy as np
    import paper_2412_11809_amd as hc
    src = tmp_path / "sizes.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "hc.h"
#define F(T, f) printf(#T "." #f " %zu\\n", offsetof(T, f));
int main(void) {
  printf("hc_hit %zu\\nhc_features %zu\\nhc_opts %zu\\nhc_server_config %zu\\nhc_completion %zu\\nhc_server_stats %zu\\n",
         sizeof(hc_hit), sizeof(hc_features), sizeof(hc_opts), sizeof(hc_server_config), sizeof(hc_completion),
         sizeof(hc_server_stats));
  F(hc_opts, stream) F(hc_server_config, hbm_budget) F(hc_server_config, flags)
  F(hc_completion, t_arrive_ns) F(hc_completion, t_final_ns)
  F(hc_server_stats, max_slots) F(hc_server_stats, final_p99) F(hc_server_stats, ns_final)
  F(hc_features, cx) F(hc_hit, tot)
  return 0;
}
""")
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)]).decode().split("\n") if line)
    got = {k: int(v) for k, v in got.items()}
    assert got["hc_hit"] == hc.HIT_DTYPE.itemsize == 16
    assert got["hc_features"] == hc.FEATURE_DTYPE.itemsize == 64
    assert got["hc_opts"] == ctypes.sizeof(hc._Opts)
    assert got["hc_server_config"] == ctypes.sizeof(hc._ServerConfig)
    assert got["hc_completion"] == hc.COMPLETION_DTYPE.itemsize
    assert got["hc_server_stats"] == ctypes.sizeof(hc._ServerStats)
    assert got["hc_opts.stream"] == hc._Opts.stream.offset
    assert got["hc_server_config.hbm_budget"] == hc._ServerConfig.hbm_budget.offset
    assert got["hc_server_config.flags"] == hc._ServerConfig.flags.offset
    assert got["hc_completion.t_arrive_ns"] == hc.COMPLETION_DTYPE.fields["t_arrive_ns"][1]
    assert got["hc_completion.t_final_ns"] == hc.COMPLETION_DTYPE.fields["t_final_ns"][1]
    assert got["hc_server_stats.max_slots"] == hc._ServerStats.max_slots.offset
    assert got["hc_server_stats.final_p99"] == hc._ServerStats.final_p99.offset
    assert got["hc_server_stats.ns_final"] == hc._ServerStats.ns_final.offset
    assert got["hc_features.cx"] == hc.FEATURE_DTYPE.fields["cx"][1]
    assert got["hc_hit.tot"] == hc.HIT_DTYPE.fields["tot"][1]


def test_server_argument_errors_are_synchronous(lib):
    import paper_2412_11809_amd as hc
    lib = hc._bind_server(lib)
    h = ctypes.c_void_p()
    c = hc._ServerConfig()
    c.n_streams = 0
    assert lib.hc_server_create(ctypes.byref(c), ctypes.byref(h)) == hc.HC_ERR_ARG
    c.n_streams, c.flags = 2, 1
    assert lib.hc_server_create(ctypes.byref(c), ctypes.byref(h)) == hc.HC_ERR_ARG
    assert lib.hc_server_create(None, ctypes.byref(h)) == hc.HC_ERR_ARG
    assert lib.hc_server_submit(None, 0, None, 0, None, 0, 0) == hc.HC_ERR_ARG
    assert lib.hc_server_flush(None, 0) == hc.HC_ERR_ARG
    k = ctypes.c_int32()
    assert lib.hc_server_poll(None, None, 0, ctypes.byref(k)) == hc.HC_ERR_ARG
    assert lib.hc_server_wait_idle(None, 10) == hc.HC_ERR_ARG
    lib.hc_server_destroy(None)
    assert hc.hc_server_now_ns() > 0
