"""Independent checkers used to pin the oracle (and, on the GPU, the library).

Nothing here shares code with ``oracle/`` or with the GPU library:

* ``brute_labels``      -- all pairs of hits, adjacency by the definition of
                           Section 2 (iii)(a), components by scipy's csgraph.
* ``window_edges``      -- every adjacent pair found by scanning the time-sorted
                           stream lag by lag (a different enumeration from the
                           oracle's per-pixel lists); used by ``partition_of``
                           and ``check_invariants``.
* ``features_from_labels`` -- the per-cluster integer features recomputed
                           directly from a labelling with numpy.
"""
import numpy as np
import scipy.sparse
import scipy.sparse.csgraph

U64 = np.uint64


def _absdiff_u64(a, b):
    a = a.astype(U64)
    b = b.astype(U64)
    return np.where(a >= b, a - b, b - a)


def canonical(comp):
    """Relabel component ids by the smallest member index."""
    comp = np.asarray(comp)
    n = comp.size
    if n == 0:
        return np.empty(0, dtype=np.int32)
    _, inv = np.unique(comp, return_inverse=True)
    mins = np.full(inv.max() + 1, n, dtype=np.int64)
    np.minimum.at(mins, inv, np.arange(n))
    return mins[inv].astype(np.int32)


def brute_labels(hits, width, height, dt):
    """O(n^2) reference: adjacency matrix from the definition, then components."""
    n = hits.shape[0]
    if n == 0:
        return np.empty(0, dtype=np.int32)
    x = hits["x"].astype(np.int64)
    y = hits["y"].astype(np.int64)
    t = hits["toa"].astype(U64)
    assert (x < width).all() and (y < height).all()
    cheb = np.maximum(np.abs(x[:, None] - x[None, :]), np.abs(y[:, None] - y[None, :]))
    td = _absdiff_u64(t[:, None], t[None, :])
    adj = (cheb <= 1) & (td <= U64(dt))
    np.fill_diagonal(adj, False)
    _, comp = scipy.sparse.csgraph.connected_components(scipy.sparse.csr_matrix(adj), directed=False)
    return canonical(comp)


def window_edges(hits, dt, max_lag=None):
    """All adjacent pairs (i, j): sort by ToA, compare each hit with the hits
    1, 2, ... positions later until no pair of that lag is within dt."""
    n = hits.shape[0]
    order = np.argsort(hits["toa"], kind="stable")
    t = hits["toa"][order].astype(U64)
    x = hits["x"][order].astype(np.int64)
    y = hits["y"][order].astype(np.int64)
    src, dst = [], []
    lag = 1
    while lag < n and (max_lag is None or lag <= max_lag):
        close = (t[lag:] - t[:-lag]) <= U64(dt)
        if not close.any():
            break
        nb = (np.abs(x[lag:] - x[:-lag]) <= 1) & (np.abs(y[lag:] - y[:-lag]) <= 1)
        sel = np.nonzero(close & nb)[0]
        src.append(order[sel])
        dst.append(order[sel + lag])
        lag += 1
    if src:
        return np.concatenate(src), np.concatenate(dst)
    return np.empty(0, np.int64), np.empty(0, np.int64)


def partition_of(hits, dt):
    """Canonical labels from the window-scan edge set."""
    n = hits.shape[0]
    if n == 0:
        return np.empty(0, dtype=np.int32)
    a, b = window_edges(hits, dt)
    g = scipy.sparse.coo_matrix((np.ones(a.size, dtype=np.int8), (a, b)), shape=(n, n)).tocsr()
    _, comp = scipy.sparse.csgraph.connected_components(g, directed=False)
    return canonical(comp)


def check_invariants(hits, labels, dt):
    """Raise AssertionError unless ``labels`` is the canonical clustering:
    a partition, label = smallest member index, every cluster connected by
    adjacent steps inside it, and no adjacent pair split across clusters."""
    n = hits.shape[0]
    labels = np.asarray(labels)
    assert labels.shape == (n,)
    if n == 0:
        return
    idx = np.arange(n)
    assert (labels >= 0).all() and (labels <= idx).all(), "label must be a member index <= i"
    assert (labels[labels] == labels).all(), "label must be its own label"
    a, b = window_edges(hits, dt)
    assert (labels[a] == labels[b]).all(), "an adjacent pair is split (not maximal)"
    # connectivity: components of the edges restricted to same-label pairs
    g = scipy.sparse.coo_matrix((np.ones(a.size, dtype=np.int8), (a, b)), shape=(n, n)).tocsr()
    _, comp = scipy.sparse.csgraph.connected_components(g, directed=False)
    assert (canonical(comp) == labels).all(), "a cluster is not connected"


def features_from_labels(hits, labels):
    """Per-cluster features in ascending label order, recomputed with numpy
    (the oracle package's numpy feature step, independent of oracle.c)."""
    import oracle
    return oracle.features_from_labels(hits, labels)


def features_equal(a, b):
    """Bit-exact comparison of two feature tables (doubles compared as bits)."""
    if a.shape != b.shape:
        return False
    for name in a.dtype.names:
        if name in ("cx", "cy"):
            if not (a[name].view(np.uint64) == b[name].view(np.uint64)).all():
                return False
        elif not (a[name] == b[name]).all():
            return False
    return True
