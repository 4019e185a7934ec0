"""Python binding of the hit-clustering library (``libhc.so``).

Thin ctypes marshalling over the C-ABI declared in ``include/hc.h``; every
step of the clustering runs in the library's HIP kernels.  PyTorch is used
only to hold device memory and to name the stream to run on.

The functions carry the C names (``hc_cluster``, ``hc_workspace_size`` ...);
``cluster`` is a convenience wrapper that allocates the outputs.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhc.so")

HC_OK = 0
HC_ERR_ARG = -1
HC_ERR_RANGE = -2
HC_ERR_WORKSPACE = -3
HC_ERR_DEVICE = -4
HC_ERR_DISORDER = -5
HC_ERR_OVERFLOW = -6
HC_ERR_BUDGET = -7
HC_ERR_BUSY = -8
DT_INFINITE = (1 << 64) - 1

# hc_hit and hc_features as numpy record types (same byte layout as hc.h)
HIT_DTYPE = np.dtype([("toa", "<u8"), ("x", "<u2"), ("y", "<u2"), ("tot", "<u2"), ("reserved", "<u2")])
FEATURE_DTYPE = np.dtype([
    ("label", "<i4"), ("size", "<u4"), ("sum_tot", "<u8"), ("toa_min", "<u8"),
    ("toa_max", "<u8"), ("sum_x_tot", "<u8"), ("sum_y_tot", "<u8"),
    ("cx", "<f8"), ("cy", "<f8"),
])


class HcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d)" % (msg, code))
        self.code = code


class _Opts(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("disorder_hint", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("stream", ctypes.c_void_p)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libhc.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhc.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_2412_11809_amd.build" % path)
    lib = ctypes.CDLL(path)
    lib.hc_workspace_size.restype = ctypes.c_size_t
    lib.hc_workspace_size.argtypes = [ctypes.POINTER(_Opts), ctypes.c_int64]
    lib.hc_cluster.restype = ctypes.c_int
    lib.hc_cluster.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Opts)]
    lib.hc_cluster_noalloc.restype = ctypes.c_int
    lib.hc_cluster_noalloc.argtypes = lib.hc_cluster.argtypes
    lib.hc_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.hc_noalloc_scratch_bytes.argtypes = []
    lib.hc_last_error.restype = ctypes.c_char_p
    lib.hc_version.restype = ctypes.c_char_p
    lib.hc_timing_enable.argtypes = [ctypes.c_int]
    lib.hc_timing_select.argtypes = [ctypes.c_char_p]
    lib.hc_timing_read.restype = ctypes.c_int
    lib.hc_timing_read.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    _lib = lib
    return lib


HC_FLAG_LINK_PIXEL_INDEX = 1
HC_FLAG_LINK_WINDOW = 2
HC_FLAG_GLOBAL_TIME = 4


def _opts(width, height, disorder_hint, workspace, stream, flags=0):
    o = _Opts()
    o.width, o.height, o.disorder_hint, o.flags = width, height, disorder_hint, flags
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if stream is not None:
        o.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return o


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check(rc):
    if rc != HC_OK:
        raise HcError(rc, load_library().hc_last_error().decode())


def hc_version():
    return load_library().hc_version().decode()


def hc_last_error():
    return load_library().hc_last_error().decode()


def hc_workspace_size(n, width=256, height=256, disorder_hint=0, flags=0):
    o = _opts(width, height, disorder_hint, None, None, flags)
    return int(load_library().hc_workspace_size(ctypes.byref(o), int(n)))


def hc_cluster(hits, n, dt, labels, features, n_clusters, width=256, height=256, disorder_hint=0,
               workspace=None, stream=None, flags=0):
    """Direct call of the C entry point on device tensors (no allocation).

    hits: uint8 tensor of n*16 bytes; labels: int32[n]; features: uint8 tensor
    of >= n*64 bytes or None; n_clusters: int32[1] (all on the GPU)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(hits.device)
    o = _opts(width, height, disorder_hint, workspace, stream, flags)
    rc = load_library().hc_cluster(_ptr(hits), int(n), int(dt), _ptr(labels), _ptr(features),
                                   _ptr(n_clusters), ctypes.byref(o))
    _check(rc)


def hc_cluster_noalloc(hits, n, dt, labels, features, n_clusters, width=256, height=256, disorder_hint=0,
                       stream=None, flags=0):
    """hc_cluster on the library's fixed scratch array (no workspace argument,
    nothing allocated); same tensors as hc_cluster."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(hits.device)
    o = _opts(width, height, disorder_hint, None, stream, flags)
    rc = load_library().hc_cluster_noalloc(_ptr(hits), int(n), int(dt), _ptr(labels), _ptr(features),
                                           _ptr(n_clusters), ctypes.byref(o))
    _check(rc)


def hc_noalloc_scratch_bytes():
    return int(load_library().hc_noalloc_scratch_bytes())


def hits_to_device(hits, device="cuda"):
    """numpy HIT_DTYPE array -> uint8 CUDA tensor (16 bytes per hit)."""
    import torch
    hits = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    return torch.from_numpy(hits.view(np.uint8).reshape(-1)).to(device)


def cluster(hits, dt, width=256, height=256, disorder_hint=0, features=True, workspace=None,
            stream=None, flags=0):
    """Cluster a device tensor of hits; returns (labels, features_bytes, n_clusters)
    as device tensors (features_bytes is uint8 [n, 64] or None)."""
    import torch
    n = hits.numel() // 16
    dev = hits.device
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    feats = torch.empty((max(n, 1), 64), dtype=torch.uint8, device=dev) if features else None
    k = torch.empty(1, dtype=torch.int32, device=dev)
    hc_cluster(hits, n, dt, labels, feats, k, width, height, disorder_hint, workspace, stream, flags)
    return labels[:n], feats, k


def features_to_numpy(feats, k):
    """Device feature bytes + count -> numpy FEATURE_DTYPE[k]."""
    k = int(k)
    if k <= 0:
        return np.empty(0, dtype=FEATURE_DTYPE)
    return feats[:k].cpu().numpy().reshape(-1).view(FEATURE_DTYPE).copy()


# ---- kernel timing (diagnostics)
def hc_timing_enable(on=True):
    load_library().hc_timing_enable(1 if on else 0)


def hc_timing_select(name=None):
    """Time only launches of kernel ``name`` (None: every kernel)."""
    load_library().hc_timing_select(name.encode() if name else None)


def hc_timing_reset():
    load_library().hc_timing_reset()


def hc_timing_read(cap=64):
    lib = load_library()
    names = (ctypes.c_char_p * cap)()
    cnt = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    k = lib.hc_timing_read(names, cnt, ms, cap)
    if k < 0:
        _check(k)
    return {names[i].decode(): (int(cnt[i]), float(ms[i])) for i in range(min(k, cap))}


# ---- stream form
def _bind_stream(lib):
    if getattr(lib, "_stream_bound", False):
        return lib
    lib.hc_stream_create.restype = ctypes.c_int
    lib.hc_stream_create.argtypes = [ctypes.POINTER(_Opts), ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.hc_stream_push.restype = ctypes.c_int
    lib.hc_stream_push.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_uint64]
    lib.hc_stream_push_ids.restype = ctypes.c_int
    lib.hc_stream_push_ids.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_uint64]
    lib.hc_stream_push_chunks.restype = ctypes.c_int
    lib.hc_stream_push_chunks.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_uint64)]
    lib.hc_stream_poll.restype = ctypes.c_int
    lib.hc_stream_poll.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.hc_stream_wait.restype = ctypes.c_int
    lib.hc_stream_wait.argtypes = [ctypes.c_void_p]
    lib.hc_stream_reserve.restype = ctypes.c_int
    lib.hc_stream_reserve.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.hc_stream_flush.restype = ctypes.c_int
    lib.hc_stream_flush.argtypes = [ctypes.c_void_p]
    lib.hc_stream_open_hits.restype = ctypes.c_int64
    lib.hc_stream_open_hits.argtypes = [ctypes.c_void_p]
    lib.hc_stream_destroy.restype = None
    lib.hc_stream_destroy.argtypes = [ctypes.c_void_p]
    lib._stream_bound = True
    return lib


class HcStream:
    """One detector stream (hc_stream_*): push device chunks (asynchronous),
    poll completions.  Chunks the device rejected are collected in
    ``rejected`` ({tag: status}) by ``poll``."""

    def __init__(self, dt, max_disorder_ticks, width=256, height=256, disorder_hint=0, stream=None, flags=0):
        import torch
        self._lib = _bind_stream(load_library())
        if stream is None:
            stream = torch.cuda.current_stream()
        self._torch_stream = stream
        o = _opts(width, height, disorder_hint, None, stream, flags)
        h = ctypes.c_void_p()
        _check(self._lib.hc_stream_create(ctypes.byref(o), int(dt), int(max_disorder_ticks), ctypes.byref(h)))
        self._h = h
        self.rejected = {}

    def hc_stream_push(self, hits, n, labels, tag):
        rc = self._lib.hc_stream_push(self._h, _ptr(hits), int(n), _ptr(labels), int(tag))
        _check(rc)

    def push(self, hits, labels, tag):
        self.hc_stream_push(hits, hits.numel() // 16, labels, tag)

    def hc_stream_push_ids(self, hits, ids, n, labels, tag):
        """hc_stream_push with caller-chosen ids (device int32[n])."""
        _check(self._lib.hc_stream_push_ids(self._h, _ptr(hits), _ptr(ids), int(n), _ptr(labels), int(tag)))

    def hc_stream_push_chunks(self, hits, counts, labels, tags):
        """k chunks back to back in the device buffer hits; labels: one device
        int32 tensor per chunk; counts and tags: sequences of k integers."""
        k = len(counts)
        c = (ctypes.c_int32 * k)(*[int(x) for x in counts])
        lp = (ctypes.c_void_p * k)(*[_ptr(x) for x in labels])
        t = (ctypes.c_uint64 * k)(*[int(x) for x in tags])
        _check(self._lib.hc_stream_push_chunks(self._h, _ptr(hits), k, c, lp, t))

    def poll(self, cap=1 << 12, closed_cap=1 << 16):
        """Tags of the chunks completed so far (rejected ones go to
        ``self.rejected``) and the closed features; drains in rounds of the caps."""
        if getattr(self, "_tags", None) is None or self._tags.size < cap or self._feats.size < closed_cap:
            import torch
            self._tags = np.empty(max(cap, 1), dtype=np.uint64)
            self._status = np.empty(max(cap, 1), dtype=np.int32)
            # pinned, so the device-to-host copy of closed features is a DMA
            self._feats_t = torch.empty(max(closed_cap, 1) * FEATURE_DTYPE.itemsize, dtype=torch.uint8,
                                        pin_memory=True)
            self._feats = self._feats_t.numpy().view(FEATURE_DTYPE)
        done, feats = [], []
        nd, nc = ctypes.c_int32(), ctypes.c_int32()
        while True:
            _check(self._lib.hc_stream_poll(self._h, self._tags.ctypes.data, self._status.ctypes.data, cap,
                                            ctypes.byref(nd), self._feats.ctypes.data, closed_cap, ctypes.byref(nc)))
            for t, s in zip(self._tags[: nd.value].tolist(), self._status[: nd.value].tolist()):
                if s == HC_OK:
                    done.append(t)
                else:
                    self.rejected[t] = s
            feats.append(self._feats[: nc.value].copy())
            if nd.value < cap and nc.value < closed_cap:
                break
        return done, np.concatenate(feats)

    def drain(self, cap=1 << 12, closed_cap=1 << 18):
        """Like ``poll``, but the closed features are only copied into the
        pinned staging buffer (and overwritten by the next call): returns the
        completed tags and the number of closed clusters drained."""
        if getattr(self, "_tags", None) is None or self._tags.size < cap or self._feats.size < closed_cap:
            import torch
            self._tags = np.empty(max(cap, 1), dtype=np.uint64)
            self._status = np.empty(max(cap, 1), dtype=np.int32)
            self._feats_t = torch.empty(max(closed_cap, 1) * FEATURE_DTYPE.itemsize, dtype=torch.uint8,
                                        pin_memory=True)
            self._feats = self._feats_t.numpy().view(FEATURE_DTYPE)
        done, n_closed = [], 0
        nd, nc = ctypes.c_int32(), ctypes.c_int32()
        while True:
            _check(self._lib.hc_stream_poll(self._h, self._tags.ctypes.data, self._status.ctypes.data, cap,
                                            ctypes.byref(nd), self._feats.ctypes.data, closed_cap, ctypes.byref(nc)))
            for t, st in zip(self._tags[: nd.value].tolist(), self._status[: nd.value].tolist()):
                if st == HC_OK:
                    done.append(t)
                else:
                    self.rejected[t] = st
            n_closed += nc.value
            if nd.value < cap and nc.value < closed_cap:
                break
        return done, n_closed

    def open_hits(self):
        """Hits held open on the device (hc_stream_open_hits)."""
        return int(self._lib.hc_stream_open_hits(self._h))

    def wait(self):
        """hc_stream_wait: every push enqueued so far has run."""
        _check(self._lib.hc_stream_wait(self._h))

    def reserve(self, max_chunk):
        _check(self._lib.hc_stream_reserve(self._h, int(max_chunk)))

    def flush(self):
        _check(self._lib.hc_stream_flush(self._h))

    def close(self):
        if self._h:
            self._lib.hc_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- batch form
def _bind_batch(lib):
    if getattr(lib, "_batch_bound", False):
        return lib
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.hc_cluster_batch.restype = ctypes.c_int
    lib.hc_cluster_batch.argtypes = [vp, i64p, ctypes.c_int32, u64p, vp, vp, vp, vp, ctypes.POINTER(_Opts)]
    lib.hc_batch_workspace_size.restype = ctypes.c_size_t
    lib.hc_batch_workspace_size.argtypes = [i64p, ctypes.c_int32, vp, ctypes.POINTER(_Opts)]
    lib.hc_batch_autotune.restype = ctypes.c_int
    lib.hc_batch_autotune.argtypes = [vp, i64p, ctypes.c_int32, u64p, vp, vp, vp, ctypes.POINTER(_Opts),
                                      ctypes.POINTER(vp)]
    lib.hc_batch_plan_describe.restype = ctypes.c_int
    lib.hc_batch_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.hc_batch_plan_destroy.restype = None
    lib.hc_batch_plan_destroy.argtypes = [vp]
    lib.hc_batch_graph_create.restype = ctypes.c_int
    lib.hc_batch_graph_create.argtypes = [vp, i64p, ctypes.c_int32, u64p, vp, vp, vp, vp, ctypes.POINTER(_Opts),
                                          ctypes.POINTER(vp)]
    lib.hc_batch_graph_launch.restype = ctypes.c_int
    lib.hc_batch_graph_launch.argtypes = [vp, vp]
    lib.hc_batch_graph_destroy.restype = None
    lib.hc_batch_graph_destroy.argtypes = [vp]
    lib._batch_bound = True
    return lib


def _batch_tables(offsets, dts):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n_chunks = len(offsets) - 1
    if np.isscalar(dts) or np.ndim(dts) == 0:
        dts = np.full(max(n_chunks, 0), int(dts), dtype=np.uint64)
    dts = np.ascontiguousarray(dts, dtype=np.uint64)
    if n_chunks < 1 or len(dts) != n_chunks:
        raise ValueError("offsets needs n_chunks + 1 entries and dts n_chunks")
    return offsets, dts, n_chunks


class BatchPlan:
    """Handle of an hc_batch_plan (from hc_batch_autotune)."""

    def __init__(self, lib, handle):
        self._lib, self._h = lib, handle

    @property
    def handle(self):
        return self._h

    def describe(self):
        buf = ctypes.create_string_buffer(256)
        _check(self._lib.hc_batch_plan_describe(self._h, buf, 256))
        return buf.value.decode()

    def close(self):
        if self._h:
            self._lib.hc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """Handle of an hc_batch_graph (captured batch launch sequence)."""

    def __init__(self, lib, handle, keep):
        self._lib, self._h, self._keep = lib, handle, keep

    def launch(self, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        _check(self._lib.hc_batch_graph_launch(self._h, s))

    def close(self):
        if self._h:
            self._lib.hc_batch_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _plan_ptr(plan):
    return None if plan is None else plan.handle


def hc_batch_workspace_size(offsets, plan=None, width=256, height=256, disorder_hint=0):
    lib = _bind_batch(load_library())
    offsets, _, n_chunks = _batch_tables(offsets, 0)
    o = _opts(width, height, disorder_hint, None, None)
    return int(lib.hc_batch_workspace_size(offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_chunks,
                                           _plan_ptr(plan), ctypes.byref(o)))


def hc_cluster_batch(hits, offsets, dts, labels, features, n_clusters, plan=None, width=256, height=256,
                     disorder_hint=0, workspace=None, stream=None, flags=0):
    """Direct call of hc_cluster_batch on device tensors; offsets/dts are host arrays."""
    import torch
    lib = _bind_batch(load_library())
    offsets, dts, n_chunks = _batch_tables(offsets, dts)
    if stream is None:
        stream = torch.cuda.current_stream(hits.device)
    o = _opts(width, height, disorder_hint, workspace, stream, flags)
    _check(lib.hc_cluster_batch(_ptr(hits), offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_chunks,
                                dts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _ptr(labels),
                                _ptr(features), _ptr(n_clusters), _plan_ptr(plan), ctypes.byref(o)))


def hc_batch_autotune(hits, offsets, dts, labels, features, n_clusters, width=256, height=256,
                      disorder_hint=0, stream=None):
    """Runs hc_batch_autotune; returns a BatchPlan (outputs hold the chosen plan's result)."""
    import torch
    lib = _bind_batch(load_library())
    offsets, dts, n_chunks = _batch_tables(offsets, dts)
    if stream is None:
        stream = torch.cuda.current_stream(hits.device)
    o = _opts(width, height, disorder_hint, None, stream)
    h = ctypes.c_void_p()
    _check(lib.hc_batch_autotune(_ptr(hits), offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_chunks,
                                 dts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _ptr(labels),
                                 _ptr(features), _ptr(n_clusters), ctypes.byref(o), ctypes.byref(h)))
    return BatchPlan(lib, h.value)


def hc_batch_graph_create(hits, offsets, dts, labels, features, n_clusters, plan=None, width=256,
                          height=256, disorder_hint=0):
    """Captures the batch launch sequence; returns a BatchGraph to replay."""
    lib = _bind_batch(load_library())
    offsets, dts, n_chunks = _batch_tables(offsets, dts)
    o = _opts(width, height, disorder_hint, None, None)
    h = ctypes.c_void_p()
    _check(lib.hc_batch_graph_create(_ptr(hits), offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     n_chunks, dts.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                     _ptr(labels), _ptr(features), _ptr(n_clusters), _plan_ptr(plan),
                                     ctypes.byref(o), ctypes.byref(h)))
    return BatchGraph(lib, h.value, (hits, labels, features, n_clusters))


def cluster_batch(hits, offsets, dts, width=256, height=256, disorder_hint=0, features=True, plan=None,
                  stream=None):
    """Cluster a batch of chunks (device hits, host offsets); returns
    (labels, features_bytes [n, 64] or None, n_clusters int32[n_chunks]) on the device."""
    import torch
    offsets, dts, n_chunks = _batch_tables(offsets, dts)
    n = int(offsets[-1])
    dev = hits.device
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    feats = torch.empty((max(n, 1), 64), dtype=torch.uint8, device=dev) if features else None
    k = torch.empty(n_chunks, dtype=torch.int32, device=dev)
    hc_cluster_batch(hits, offsets, dts, labels, feats, k, plan, width, height, disorder_hint, None, stream)
    return labels[:n], feats, k


# ---- per-cluster products
BOX_DTYPE = np.dtype([("x_min", "<u2"), ("x_max", "<u2"), ("y_min", "<u2"), ("y_max", "<u2")])


class _Filter(ctypes.Structure):
    _fields_ = [("min_size", ctypes.c_uint32), ("max_size", ctypes.c_uint32),
                ("min_sum_tot", ctypes.c_uint64), ("max_sum_tot", ctypes.c_uint64),
                ("toa_from", ctypes.c_uint64), ("toa_to", ctypes.c_uint64)]


def _bind_products(lib):
    if getattr(lib, "_products_bound", False):
        return lib
    vp = ctypes.c_void_p
    lib.hc_products_workspace_size.restype = ctypes.c_size_t
    lib.hc_products_workspace_size.argtypes = [ctypes.c_int64]
    lib.hc_cluster_products.restype = ctypes.c_int
    lib.hc_cluster_products.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.POINTER(_Filter), vp, vp, vp, vp, vp,
                                        vp, vp, ctypes.c_size_t, vp]
    lib._products_bound = True
    return lib


def hc_products_workspace_size(n):
    return int(_bind_products(load_library()).hc_products_workspace_size(int(n)))


def hc_cluster_products(hits, n, labels, features, n_clusters, keep_rows, n_keep, boxes=None, grouped=None,
                        grouped_idx=None, row_start=None, filter=None, workspace=None, stream=None):
    """Direct call of hc_cluster_products on device tensors.  filter: None or
    a dict with any of min_size, max_size, min_sum_tot, max_sum_tot,
    toa_from, toa_to."""
    import torch
    lib = _bind_products(load_library())
    if stream is None:
        stream = torch.cuda.current_stream(labels.device)
    f = None
    if filter is not None:
        f = _Filter(0, 0xFFFFFFFF, 0, (1 << 64) - 1, 0, (1 << 64) - 1)
        for k, v in filter.items():
            setattr(f, k, int(v))
    if workspace is None:
        workspace = torch.empty(max(1, hc_products_workspace_size(n)), dtype=torch.uint8, device=labels.device)
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _check(lib.hc_cluster_products(_ptr(hits), int(n), _ptr(labels), _ptr(features), _ptr(n_clusters),
                                   ctypes.byref(f) if f is not None else None, _ptr(boxes), _ptr(keep_rows),
                                   _ptr(n_keep), _ptr(grouped), _ptr(grouped_idx), _ptr(row_start),
                                   _ptr(workspace), workspace.numel(), s))
    return workspace


# ---- host ingest front end
class _IngestConfig(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32), ("disorder_hint", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("dt", ctypes.c_uint64), ("max_disorder_ticks", ctypes.c_uint64),
                ("t_closing", ctypes.c_uint64), ("buffer_hits", ctypes.c_int32), ("reserve_hits", ctypes.c_int32),
                ("n_buffers", ctypes.c_int32), ("reserved", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class _IngestStats(ctypes.Structure):
    _fields_ = [("hits_fed", ctypes.c_int64), ("hits_done", ctypes.c_int64), ("buffers_sent", ctypes.c_int64),
                ("buffers_done", ctypes.c_int64), ("forced_sends", ctypes.c_int64), ("diverted", ctypes.c_int64),
                ("waits", ctypes.c_int64)]


def _bind_ingest(lib):
    if getattr(lib, "_ingest_bound", False):
        return lib
    vp = ctypes.c_void_p
    lib.hc_ingest_create.restype = ctypes.c_int
    lib.hc_ingest_create.argtypes = [ctypes.POINTER(_IngestConfig), vp, ctypes.c_int64, ctypes.POINTER(vp)]
    lib.hc_ingest_feed.restype = ctypes.c_int
    lib.hc_ingest_feed.argtypes = [vp, vp, ctypes.c_int64]
    lib.hc_ingest_finish.restype = ctypes.c_int
    lib.hc_ingest_finish.argtypes = [vp]
    lib.hc_ingest_stats_read.restype = ctypes.c_int
    lib.hc_ingest_stats_read.argtypes = [vp, ctypes.POINTER(_IngestStats)]
    lib.hc_ingest_destroy.restype = None
    lib.hc_ingest_destroy.argtypes = [vp]
    lib._ingest_bound = True
    return lib


class HcIngest:
    """Host ingest front end (hc_ingest_*): feed host hits in arrival order;
    labels land in ``labels`` (a host int32 array, indexed by arrival)."""

    def __init__(self, labels, dt, max_disorder_ticks, t_closing, buffer_hits, reserve_hits, width=256,
                 height=256, disorder_hint=0, n_buffers=0, stream=None):
        import torch
        self._lib = _bind_ingest(load_library())
        if stream is None:
            stream = torch.cuda.current_stream()
        c = _IngestConfig()
        c.width, c.height, c.disorder_hint, c.flags = width, height, disorder_hint, 0
        c.dt, c.max_disorder_ticks, c.t_closing = int(dt), int(max_disorder_ticks), int(t_closing)
        c.buffer_hits, c.reserve_hits, c.n_buffers, c.reserved = int(buffer_hits), int(reserve_hits), n_buffers, 0
        c.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self._labels = labels
        h = ctypes.c_void_p()
        _check(self._lib.hc_ingest_create(ctypes.byref(c), _host_ptr(labels), _host_len(labels, 4),
                                          ctypes.byref(h)))
        self._h = h

    def feed(self, hits):
        """hits: host HIT_DTYPE array (or uint8 tensor of 16-byte records)."""
        _check(self._lib.hc_ingest_feed(self._h, _host_ptr(hits), _host_len(hits, 16)))

    def finish(self):
        _check(self._lib.hc_ingest_finish(self._h))

    def stats(self):
        s = _IngestStats()
        _check(self._lib.hc_ingest_stats_read(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _IngestStats._fields_}

    def close(self):
        if self._h:
            self._lib.hc_ingest_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- served form
class _ServerConfig(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32), ("n_streams", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("dt", ctypes.c_uint64), ("max_disorder_ticks", ctypes.c_uint64),
                ("hbm_budget", ctypes.c_uint64), ("disorder_hint", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("max_chunk_hits", ctypes.c_int32), ("reserved", ctypes.c_int32)]


COMPLETION_DTYPE = np.dtype([
    ("tag", "<u8"), ("stream_id", "<i4"), ("status", "<i4"), ("n_hits", "<i4"), ("n_closed", "<i4"),
    ("t_arrive_ns", "<u8"), ("t_admit_ns", "<u8"), ("t_processed_ns", "<u8"), ("t_final_ns", "<u8"),
])


class _ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("hits_completed", ctypes.c_int64), ("queued", ctypes.c_int64), ("pending_final", ctypes.c_int64),
                ("hbm_budget", ctypes.c_uint64), ("hbm_in_use", ctypes.c_uint64), ("hbm_peak", ctypes.c_uint64),
                ("max_slots", ctypes.c_int32), ("peak_slots_in_use", ctypes.c_int32),
                ("processing_p50", ctypes.c_uint64), ("processing_p99", ctypes.c_uint64),
                ("final_p50", ctypes.c_uint64), ("final_p99", ctypes.c_uint64),
                ("ns_admit_wait", ctypes.c_uint64), ("ns_push", ctypes.c_uint64), ("ns_drain", ctypes.c_uint64),
                ("ns_final", ctypes.c_uint64), ("pushes", ctypes.c_int64)]


def _bind_server(lib):
    if getattr(lib, "_server_bound", False):
        return lib
    vp = ctypes.c_void_p
    lib.hc_server_now_ns.restype = ctypes.c_uint64
    lib.hc_server_now_ns.argtypes = []
    lib.hc_server_create.restype = ctypes.c_int
    lib.hc_server_create.argtypes = [ctypes.POINTER(_ServerConfig), ctypes.POINTER(vp)]
    lib.hc_server_submit.restype = ctypes.c_int
    lib.hc_server_submit.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, vp, ctypes.c_uint64, ctypes.c_uint64]
    lib.hc_server_flush.restype = ctypes.c_int
    lib.hc_server_flush.argtypes = [vp, ctypes.c_int32]
    lib.hc_server_poll.restype = ctypes.c_int
    lib.hc_server_poll.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.hc_server_closed.restype = ctypes.c_int
    lib.hc_server_closed.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.hc_server_wait_idle.restype = ctypes.c_int
    lib.hc_server_wait_idle.argtypes = [vp, ctypes.c_int32]
    lib.hc_server_stats_read.restype = ctypes.c_int
    lib.hc_server_stats_read.argtypes = [vp, ctypes.POINTER(_ServerStats)]
    lib.hc_server_destroy.restype = None
    lib.hc_server_destroy.argtypes = [vp]
    lib._server_bound = True
    return lib


def hc_server_now_ns():
    return int(_bind_server(load_library()).hc_server_now_ns())


class HcServer:
    """Served form (hc_server_*): submit host chunks of several detector
    streams; the library admits them by slot and HBM budget and overlaps their
    device work.  Host buffers must stay alive until their completion is polled
    (this wrapper keeps a reference until then)."""

    def __init__(self, n_streams, dt, max_disorder_ticks, width=256, height=256, max_slots=0,
                 hbm_budget=0, disorder_hint=0, max_chunk_hits=0):
        self._lib = _bind_server(load_library())
        c = _ServerConfig()
        c.width, c.height, c.n_streams, c.max_slots = width, height, n_streams, max_slots
        c.dt, c.max_disorder_ticks, c.hbm_budget = int(dt), int(max_disorder_ticks), int(hbm_budget)
        c.disorder_hint, c.flags = disorder_hint, 0
        c.max_chunk_hits, c.reserved = int(max_chunk_hits), 0
        h = ctypes.c_void_p()
        _check(self._lib.hc_server_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def hc_server_submit(self, stream_id, hits, n, labels, tag, t_arrive_ns):
        _check(self._lib.hc_server_submit(self._h, int(stream_id), hits, int(n), labels, int(tag),
                                          int(t_arrive_ns)))

    def submit(self, stream_id, hits, labels, tag, t_arrive_ns=None):
        """hits: host HIT_DTYPE array (pinned or pageable); labels: host int32 array."""
        if t_arrive_ns is None:
            t_arrive_ns = hc_server_now_ns()
        hp, lp = _host_ptr(hits), _host_ptr(labels)
        n = _host_len(hits, 16)
        self._keep[(int(stream_id), int(tag))] = (hits, labels)
        try:
            self.hc_server_submit(stream_id, hp, n, lp, tag, t_arrive_ns)
        except Exception:
            self._keep.pop((int(stream_id), int(tag)), None)
            raise

    def flush(self, stream_id):
        _check(self._lib.hc_server_flush(self._h, int(stream_id)))

    def poll(self, cap=4096):
        out = np.empty(max(cap, 1), dtype=COMPLETION_DTYPE)
        k = ctypes.c_int32()
        _check(self._lib.hc_server_poll(self._h, out.ctypes.data, cap, ctypes.byref(k)))
        out = out[: k.value].copy()
        for c in out:
            self._keep.pop((int(c["stream_id"]), int(c["tag"])), None)
        return out

    def closed(self, stream_id, cap=1 << 20):
        out = np.empty(max(cap, 1), dtype=FEATURE_DTYPE)
        k = ctypes.c_int32()
        _check(self._lib.hc_server_closed(self._h, int(stream_id), out.ctypes.data, cap, ctypes.byref(k)))
        return out[: k.value].copy()

    def closed_into(self, stream_id, out):
        """Closed features of one stream into ``out`` (a FEATURE_DTYPE array,
        reused by the caller); returns how many were written."""
        assert out.dtype == FEATURE_DTYPE and out.flags["C_CONTIGUOUS"]
        k = ctypes.c_int32()
        _check(self._lib.hc_server_closed(self._h, int(stream_id), out.ctypes.data, int(out.size), ctypes.byref(k)))
        return k.value

    def wait_idle(self, timeout_ms=60000):
        _check(self._lib.hc_server_wait_idle(self._h, int(timeout_ms)))

    def stats(self):
        s = _ServerStats()
        _check(self._lib.hc_server_stats_read(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if self._h:
            self._lib.hc_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_ptr(a):
    if hasattr(a, "data_ptr"):
        assert not a.is_cuda, "server buffers live in host memory"
        return a.data_ptr()
    return a.ctypes.data


def _host_len(a, item):
    if hasattr(a, "data_ptr"):
        return a.numel() * a.element_size() // item
    return a.nbytes // item
