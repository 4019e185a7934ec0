"""Parity oracle for the hit clusterer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

``cluster`` wraps ``oracle.c`` (plain sequential C: time sort, per-pixel lists,
breadth-first search over the adjacency relation of the paper's Section 2
(iii)(a), then exact integer features).  ``cluster_global`` wraps
``oracle_global.c``, the clusters of the Section 2 (iii)(b) variant (parts
refined by ToA gaps and spatial components until stable), with the features
recomputed from its labels by ``features_from_labels`` (numpy).  The shared
object is compiled with gcc on first use (or by ``build()``).
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_GLOBAL = os.path.join(_HERE, "oracle_global.c")
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
    """Compile the C oracle with gcc (-O2, no fast-math); the default build
    also holds the (iii)(b) clusterer."""
    srcs = [src] + ([_SRC_GLOBAL] if src == _SRC else [])
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", out] + srcs)
    return out


def load(path=None):
    """Load (building if absent) the oracle shared object."""
    global _lib
    with _lock:
        if path is not None:
            return _bind(ctypes.CDLL(path))
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                        os.path.getmtime(_SRC_GLOBAL)):
                build()
            _lib = _bind(ctypes.CDLL(_LIB))
        return _lib


def _bind(lib):
    lib.oracle_cluster.restype = ctypes.c_int
    lib.oracle_cluster.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_int64)]
    if hasattr(lib, "oracle_cluster_global"):
        lib.oracle_cluster_global.restype = ctypes.c_int64
        lib.oracle_cluster_global.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_uint64, ctypes.c_void_p]
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


def features_from_labels(hits, labels):
    """Per-cluster features (size, ToT sum, ToA min/max, x*ToT and y*ToT sums,
    centroid) in ascending label order, computed with numpy from given labels;
    the same definitions as the feature step of oracle.c."""
    labels = np.asarray(labels, dtype=np.int64)
    U64 = np.uint64
    roots = np.unique(labels)
    inv = np.searchsorted(roots, labels)
    k = roots.size
    out = np.zeros(k, dtype=FEATURE_DTYPE)
    out["label"] = roots
    x = hits["x"].astype(U64)
    y = hits["y"].astype(U64)
    tot = hits["tot"].astype(U64)
    toa = hits["toa"].astype(U64)
    size = np.zeros(k, np.int64)
    np.add.at(size, inv, 1)
    st = np.zeros(k, U64); np.add.at(st, inv, tot)
    sxt = np.zeros(k, U64); np.add.at(sxt, inv, x * tot)
    syt = np.zeros(k, U64); np.add.at(syt, inv, y * tot)
    sx = np.zeros(k, U64); np.add.at(sx, inv, x)
    sy = np.zeros(k, U64); np.add.at(sy, inv, y)
    tmin = np.full(k, np.iinfo(U64).max, U64); np.minimum.at(tmin, inv, toa)
    tmax = np.zeros(k, U64); np.maximum.at(tmax, inv, toa)
    out["size"] = size
    out["sum_tot"] = st
    out["toa_min"] = tmin
    out["toa_max"] = tmax
    out["sum_x_tot"] = sxt
    out["sum_y_tot"] = syt
    w = st > 0
    out["cx"] = np.where(w, sxt.astype(np.float64) / np.maximum(st, 1).astype(np.float64),
                         sx.astype(np.float64) / size.astype(np.float64))
    out["cy"] = np.where(w, syt.astype(np.float64) / np.maximum(st, 1).astype(np.float64),
                         sy.astype(np.float64) / size.astype(np.float64))
    return out


def cluster_global(hits, width=256, height=256, dt=128, features=True, lib=None):
    """Clusters of the Section 2 (iii)(b) variant: ``(labels int32[n],
    features FEATURE_DTYPE[K])`` with the same conventions as ``cluster``."""
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    n = hits.shape[0]
    lib = lib or load()
    labels = np.empty(n, dtype=np.int32)
    k = lib.oracle_cluster_global(hits.ctypes.data if n else None, n, width, height, int(dt),
                                  labels.ctypes.data if n else None)
    if k == -2:
        raise OracleRangeError("hit outside the %dx%d sensor" % (width, height))
    if k < 0:
        raise RuntimeError("oracle_cluster_global failed with status %d" % k)
    if not features:
        return labels, int(k)
    f = features_from_labels(hits, labels) if n else np.empty(0, dtype=FEATURE_DTYPE)
    assert f.size == k
    return labels, f
