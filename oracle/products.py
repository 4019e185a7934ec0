"""Per-cluster products of a clustering -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` may import this module; the product library never loads it.
Given hits, their labels and the feature table (rows in ascending label
order), it computes what the paper names around the clustering itself:

  * bounding box of every cluster: the smallest sensor-aligned rectangle
    that encloses all of its hits (Section 3.3, second step of the merge
    test: boxes of two clusters that do not intersect rule out a merge);
  * filtering of the cluster output to reduce the data volume (Section 3.1,
    cluster outputting; Section 6 lists filtering among the tasks to move to
    the GPU): a cluster is kept when its size, ToT sum and first ToA lie in
    closed ranges;
  * the hits of the kept clusters grouped cluster by cluster, so that the
    hits of one cluster form one block of memory (step 6 of the paper's
    high-level GPU algorithm); clusters in ascending label order, hits of one
    cluster in ascending input index.

Plain numpy, each step a direct transcription of the definition above.
"""
import numpy as np

BOX_DTYPE = np.dtype([("x_min", "<u2"), ("x_max", "<u2"), ("y_min", "<u2"), ("y_max", "<u2")])

U32MAX = (1 << 32) - 1
U64MAX = (1 << 64) - 1


def boxes(hits, labels, features):
    """BOX_DTYPE[K]: box of feature row k = min/max of x and y over the hits
    whose label equals features[k]['label']."""
    K = features.size
    out = np.empty(K, dtype=BOX_DTYPE)
    if K == 0:
        return out
    row = np.searchsorted(features["label"], labels)  # labels are feature labels
    assert np.array_equal(features["label"][row], labels), "every label must have a feature row"
    x = hits["x"].astype(np.int64)
    y = hits["y"].astype(np.int64)
    for f, init, op in (("x_min", 1 << 20, np.minimum), ("x_max", -1, np.maximum),
                        ("y_min", 1 << 20, np.minimum), ("y_max", -1, np.maximum)):
        acc = np.full(K, init, dtype=np.int64)
        op.at(acc, row, x if f[0] == "x" else y)
        out[f] = acc
    return out


def keep_rows(features, min_size=0, max_size=U32MAX, min_sum_tot=0, max_sum_tot=U64MAX,
              toa_from=0, toa_to=U64MAX):
    """Ascending indices of the feature rows that pass every closed range."""
    f = features
    ok = ((f["size"] >= min_size) & (f["size"] <= max_size) &
          (f["sum_tot"] >= np.uint64(min_sum_tot)) & (f["sum_tot"] <= np.uint64(max_sum_tot)) &
          (f["toa_min"] >= np.uint64(toa_from)) & (f["toa_min"] <= np.uint64(toa_to)))
    return np.nonzero(ok)[0].astype(np.int32)


def grouped(labels, features, rows):
    """(hit indices of the kept clusters, cluster by cluster; start of every
    kept cluster's block, len(rows) + 1 entries).  A stable sort of the hits
    by the position of their cluster among the kept rows (dropped clusters
    last) puts every kept cluster in one block, hits in input order."""
    K = features.size
    rank = np.full(K + 1, rows.size, dtype=np.int64)  # dropped rows sort behind every kept one
    rank[rows] = np.arange(rows.size)
    row = np.searchsorted(features["label"], labels) if labels.size else np.empty(0, dtype=np.int64)
    key = rank[row]
    order = np.argsort(key, kind="stable")
    sizes = features["size"][rows].astype(np.int64)
    start = np.zeros(rows.size + 1, dtype=np.int64)
    start[1:] = np.cumsum(sizes)
    return order[: start[-1]].astype(np.int32), start
