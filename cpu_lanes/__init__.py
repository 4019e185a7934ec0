"""Multi-lane CPU clustering (the paper's CPU method, Section 3): a comparison
baseline for the GPU library, used by bench.py and the tests only.

``lanes.cpp`` is compiled with g++ (-O2, threads) into ``liblanes.so`` on
first use or by ``build()``.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lanes.cpp")
_LIB = os.path.join(_HERE, "liblanes.so")
_lock = threading.Lock()
_lib = None


def build():
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-Wall", "-o", _LIB, _SRC])
    return _LIB


def load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_LIB)
            lib.lanes_cluster.restype = ctypes.c_int64
            lib.lanes_cluster.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p]
            _lib = lib
        return _lib


def cluster(hits, width, height, dt, lanes, window_ticks):
    """labels int32[n] (smallest input index of each cluster) and the count."""
    hits = np.ascontiguousarray(hits)
    assert hits.dtype.itemsize == 16
    n = hits.shape[0]
    labels = np.empty(n, dtype=np.int32)
    k = load().lanes_cluster(hits.ctypes.data if n else None, n, width, height, int(dt), int(lanes),
                             int(window_ticks), labels.ctypes.data if n else None)
    if k < 0:
        raise ValueError("lanes_cluster failed with status %d" % k)
    return labels, int(k)
