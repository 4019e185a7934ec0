"""Parity oracle for the hit clusterer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

``cluster`` wraps ``oracle.c`` (plain sequential C: time sort, per-pixel lists,
breadth-first search over the adjacency relation of the paper's Section 2
(iii)(a), then exact integer features).  The shared object is compiled with gcc
on first use (or by ``build()``).
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Record layouts of the paper's pixel hit (Section 1: x, y, ToA, ToT) and of
# the per-cluster feature record.  Kept here, independent of the GPU library.
HIT_DTYPE = np.dtype([("toa", "<u8"), ("x", "<u2"), ("y", "<u2"), ("tot", "<u2"), ("reserved", "<u2")])
FEATURE_DTYPE = np.dtype([
    ("label", "<i4"), ("size", "<u4"), ("sum_tot", "<u8"), ("toa_min", "<u8"),
    ("toa_max", "<u8"), ("sum_x_tot", "<u8"), ("sum_y_tot", "<u8"),
    ("cx", "<f8"), ("cy", "<f8"),
])
assert HIT_DTYPE.itemsize == 16 and FEATURE_DTYPE.itemsize == 64

DT_INFINITE = (1 << 64) - 1


def build(src=_SRC, out=_LIB):
    """Compile the C oracle with gcc (-O2, no fast-math)."""
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", out, src])
    return out


def load(path=None):
    """Load (building if absent) the oracle shared object."""
    global _lib
    with _lock:
        if path is not None:
            return _bind(ctypes.CDLL(path))
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = _bind(ctypes.CDLL(_LIB))
        return _lib


def _bind(lib):
    lib.oracle_cluster.restype = ctypes.c_int
    lib.oracle_cluster.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_int64)]
    return lib


class OracleRangeError(ValueError):
    """A hit lies outside the sensor."""


def cluster(hits, width=256, height=256, dt=128, features=True, lib=None):
    """Cluster ``hits`` (structured array of HIT_DTYPE).

    Returns ``(labels int32[n], features FEATURE_DTYPE[K])``; ``labels[i]`` is
    the smallest input index in hit i's cluster and ``features`` lists the
    clusters in ascending label order.
    """
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    n = hits.shape[0]
    lib = lib or load()
    labels = np.empty(n, dtype=np.int32)
    feats = np.empty(n if features else 0, dtype=FEATURE_DTYPE)
    k = ctypes.c_int64(0)
    rc = lib.oracle_cluster(hits.ctypes.data if n else None, n, width, height, int(dt),
                            labels.ctypes.data if n else None,
                            feats.ctypes.data if (features and n) else None, ctypes.byref(k))
    if rc == -2:
        raise OracleRangeError("hit outside the %dx%d sensor" % (width, height))
    if rc != 0:
        raise RuntimeError("oracle_cluster failed with status %d" % rc)
    return labels, feats[: k.value] if features else k.value
