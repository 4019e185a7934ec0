"""Pins of the per-cluster product oracle (oracle/products.py) against
brute force over pure-Python loops on small inputs, and against what the
definitions fix in closed form: the box of one hit, of a straight track, and
of a cluster spanning the sensor; filters that keep everything or nothing;
and grouping as a permutation whose blocks are exactly the kept clusters."""
import numpy as np
import pytest

import hitgen
import oracle
from oracle import products

U64 = (1 << 64) - 1


def brute_boxes(hits, labels):
    box = {}
    for i in range(hits.size):
        x, y, lab = int(hits["x"][i]), int(hits["y"][i]), int(labels[i])
        b = box.get(lab)
        box[lab] = (x, x, y, y) if b is None else (min(b[0], x), max(b[1], x), min(b[2], y), max(b[3], y))
    return box


@pytest.mark.parametrize("seed", range(40))
def test_boxes_match_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    hits = hitgen.uniform_hits(n, seed, width=int(rng.integers(1, 20)), height=int(rng.integers(1, 20)),
                               toa_hi=int(rng.integers(1, 200)))
    labels, feats = oracle.cluster(hits, 256, 256, int(rng.integers(0, 20)))
    got = products.boxes(hits, labels, feats)
    want = brute_boxes(hits, labels)
    assert len(want) == feats.size
    for k in range(feats.size):
        assert tuple(int(v) for v in got[k]) == want[int(feats["label"][k])]


def test_box_closed_forms():
    hits = np.zeros(3, dtype=hitgen.HIT_DTYPE)
    # one isolated hit: a degenerate box on its pixel
    hits[0] = (5, 7, 9, 1, 0)
    # a horizontal track of 2 hits far away
    hits[1] = (1000, 100, 50, 1, 0)
    hits[2] = (1001, 101, 50, 1, 0)
    labels, feats = oracle.cluster(hits, 256, 256, 10)
    b = products.boxes(hits, labels, feats)
    assert tuple(b[0]) == (7, 7, 9, 9)
    assert tuple(b[1]) == (100, 101, 50, 50)
    # a diagonal staircase across the whole sensor, all at one ToA
    m = 64
    h = np.zeros(m, dtype=hitgen.HIT_DTYPE)
    h["x"] = np.arange(m)
    h["y"] = np.arange(m)[::-1]
    labels, feats = oracle.cluster(h, 64, 64, 0)
    assert feats.size == 1
    assert tuple(products.boxes(h, labels, feats)[0]) == (0, 63, 0, 63)


def test_every_hit_inside_its_box_and_edges_attained():
    hits, p = hitgen.mixed_10m(n=60_000, seed=5)
    labels, feats = oracle.cluster(hits, 256, 256, p["dt"])
    b = products.boxes(hits, labels, feats)
    row = np.searchsorted(feats["label"], labels)
    assert (hits["x"] >= b["x_min"][row]).all() and (hits["x"] <= b["x_max"][row]).all()
    assert (hits["y"] >= b["y_min"][row]).all() and (hits["y"] <= b["y_max"][row]).all()
    for f, col in (("x_min", "x"), ("x_max", "x"), ("y_min", "y"), ("y_max", "y")):
        hit_on_edge = np.zeros(feats.size, dtype=bool)
        hit_on_edge[row[hits[col] == b[f][row]]] = True
        assert hit_on_edge.all(), f


def test_filter_closed_forms():
    hits, p = hitgen.blobs_100k(n=20_000, seed=3)
    labels, feats = oracle.cluster(hits, 256, 256, p["dt"])
    K = feats.size
    assert np.array_equal(products.keep_rows(feats), np.arange(K))
    assert products.keep_rows(feats, min_size=2, max_size=1).size == 0
    singles = products.keep_rows(feats, max_size=1)
    assert np.array_equal(singles, np.nonzero(feats["size"] == 1)[0])
    # brute force over the rows
    lo, hi = 100, 5000
    t0 = int(np.median(feats["toa_min"]))
    want = [k for k in range(K) if 2 <= feats["size"][k] <= 30 and lo <= feats["sum_tot"][k] <= hi and
            feats["toa_min"][k] >= t0]
    got = products.keep_rows(feats, min_size=2, max_size=30, min_sum_tot=lo, max_sum_tot=hi, toa_from=t0)
    assert got.tolist() == want


def test_grouping_matches_a_loop_over_the_kept_clusters():
    for seed in range(10):
        hits = hitgen.uniform_hits(400, 70 + seed, width=12, height=12, toa_hi=300)
        labels, feats = oracle.cluster(hits, 256, 256, 5)
        rows = products.keep_rows(feats, min_size=1 + seed % 3)
        idx, start = products.grouped(labels, feats, rows)
        want, at = [], [0]
        for k in rows:  # brute force: every kept cluster's members, in input order
            members = [i for i in range(hits.size) if labels[i] == feats["label"][k]]
            want += members
            at.append(at[-1] + len(members))
        assert idx.tolist() == want and start.tolist() == at


def test_grouping_is_the_kept_clusters_in_blocks():
    hits, p = hitgen.mixed_10m(n=30_000, seed=9)
    labels, feats = oracle.cluster(hits, 256, 256, p["dt"])
    rows = products.keep_rows(feats, min_size=3)
    idx, start = products.grouped(labels, feats, rows)
    assert start[-1] == idx.size == int(feats["size"][rows].sum())
    assert np.array_equal(np.diff(start), feats["size"][rows].astype(np.int64))
    assert np.unique(idx).size == idx.size
    for j, k in enumerate(rows):
        block = idx[start[j]:start[j + 1]]
        assert (labels[block] == feats["label"][k]).all()
        assert (np.diff(block) > 0).all()  # input order inside a cluster
        assert block[0] == feats["label"][k]  # the label is the smallest index
