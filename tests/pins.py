"""Pins of the oracle: checks against what the paper and mathematics fix.

Each ``pin_*`` takes the oracle's loaded shared object (so the mutation tests
can run the same checks against deliberately broken oracles) and raises
``AssertionError`` on any disagreement.  None of them re-uses the oracle's
code: the references are the hand-derived fixtures in ``tests/golden``,
all-pairs brute force, scipy's image labelling, closed forms, metamorphic
relations and the independent invariant checker in ``refs.py``.
"""
import glob
import os

import numpy as np
import scipy.ndimage

import hitgen
import oracle
from refs import (brute_labels, canonical, check_invariants, features_equal,
                  features_from_labels, partition_of)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U64MAX = (1 << 64) - 1


def make_hits(rows):
    rows = list(rows)
    h = np.zeros(len(rows), dtype=oracle.HIT_DTYPE)
    for i, r in enumerate(rows):
        h[i]["x"], h[i]["y"], h[i]["toa"] = r[0], r[1], r[2]
        h[i]["tot"] = r[3] if len(r) > 3 else 1
    return h


def load_golden(path):
    """Parse one fixture: returns (width, height, dt, hits, labels, feature rows)."""
    head, rows, labels, feats = None, [], [], []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if head is None:
            head = tuple(int(v) for v in tok)
        elif tok[0] == "F":
            feats.append(tok[1:])
        else:
            rows.append(tuple(int(v) for v in tok[:4]))
            labels.append(int(tok[4]))
    w, h, dt = head
    return w, h, dt, make_hits(rows), np.array(labels, dtype=np.int32), feats


def pin_golden(lib):
    files = sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))
    files = [f for f in files if not f.endswith("README.txt")]
    assert files
    for path in files:
        w, h, dt, hits, want, feats = load_golden(path)
        got, f = oracle.cluster(hits, w, h, dt, lib=lib)
        assert (got == want).all(), "%s: labels %s, expected %s" % (os.path.basename(path), got, want)
        for row in feats:
            lab = int(row[0])
            rec = f[f["label"] == lab]
            assert rec.size == 1, path
            rec = rec[0]
            ints = [int(v) for v in row[1:7]]
            assert [int(rec[k]) for k in ("size", "sum_tot", "toa_min", "toa_max", "sum_x_tot",
                                          "sum_y_tot")] == ints, (path, rec)
            assert rec["cx"] == float(row[7]) and rec["cy"] == float(row[8]), (path, rec)


def pin_bruteforce(lib, cases=300, seed=7):
    rng = np.random.default_rng(seed)
    for c in range(cases):
        n = int(rng.integers(0, 61))
        w = int(rng.integers(1, 7))
        hh = int(rng.integers(1, 7))
        span = int(rng.integers(1, 300))
        hits = hitgen.uniform_hits(n, [seed, c], w, hh, span,
                                   disorder=None if c % 3 else int(rng.integers(0, 8)))
        dt = [0, 1, 5, 20, 64, 150, U64MAX][int(rng.integers(0, 7))]
        got, _ = oracle.cluster(hits, w, hh, dt, lib=lib)
        want = brute_labels(hits, w, hh, dt)
        assert (got == want).all(), "case %d n=%d %dx%d dt=%d" % (c, n, w, hh, dt)


def pin_image_labelling(lib, seed=11):
    """dt = infinity and distinct pixels: clusters are exactly the 8-connected
    components of the binary image (scipy.ndimage.label, 3x3 structure)."""
    rng = np.random.default_rng(seed)
    for w, hh, dens in [(40, 30, 0.35), (64, 64, 0.45), (17, 90, 0.5), (256, 256, 0.1)]:
        img = rng.random((hh, w)) < dens
        ys, xs = np.nonzero(img)
        perm = rng.permutation(xs.size)
        xs, ys = xs[perm], ys[perm]
        hits = make_hits(zip(xs, ys, rng.integers(0, 1 << 40, xs.size)))
        got, _ = oracle.cluster(hits, w, hh, U64MAX, lib=lib)
        lab, _ = scipy.ndimage.label(img, structure=np.ones((3, 3), dtype=int))
        want = canonical(lab[ys, xs])
        assert (got == want).all(), (w, hh)


def pin_closed_forms(lib, seed=13):
    rng = np.random.default_rng(seed)
    # n = 0 and n = 1
    got, f = oracle.cluster(make_hits([]), 256, 256, 5, lib=lib)
    assert got.size == 0 and f.size == 0
    got, f = oracle.cluster(make_hits([(3, 4, 99, 7)]), 256, 256, 5, lib=lib)
    assert list(got) == [0] and f.size == 1 and f[0]["cx"] == 3.0 and f[0]["cy"] == 4.0
    # all hits on one pixel: clusters are the runs between ToA gaps > dt
    for trial in range(20):
        n = int(rng.integers(1, 200))
        t = np.sort(rng.integers(0, 2000, n))
        dt = int(rng.integers(0, 40))
        perm = rng.permutation(n)
        hits = make_hits([(7, 9, int(v)) for v in t[perm]])
        got, _ = oracle.cluster(hits, 16, 16, dt, lib=lib)
        run = np.concatenate([[0], np.cumsum(np.diff(t) > dt)])   # run id in time order
        want = canonical(run[perm])
        assert (got == want).all()
        assert np.unique(got).size == 1 + int((np.diff(t) > dt).sum())
    # straight 8-connected track: 1 + number of consecutive gaps > dt
    for trial in range(20):
        L = int(rng.integers(2, 120))
        dx, dy = [(1, 0), (0, 1), (1, 1), (1, -1)][trial % 4]
        x0, y0 = 5, 130
        steps = rng.integers(0, 30, L)
        steps[0] = 0
        t = np.cumsum(steps) + 1000
        dt = int(rng.integers(0, 30))
        pts = [(x0 + k * dx, y0 + k * dy, int(t[k])) for k in range(L)]
        perm = rng.permutation(L)
        hits = make_hits([pts[p] for p in perm])
        got, _ = oracle.cluster(hits, 256, 256, dt, lib=lib)
        assert np.unique(got).size == 1 + int((np.diff(t) > dt).sum())
    # dt = 0: only equal-ToA neighbours join
    hits = make_hits([(1, 1, 5), (2, 2, 5), (3, 3, 6), (3, 3, 6), (4, 4, 7)])
    got, _ = oracle.cluster(hits, 8, 8, 0, lib=lib)
    assert list(got) == [0, 0, 2, 2, 4]
    # isolated hits (pixels at least two apart) are all singletons
    hits = make_hits([(2 * i, 2 * j, i * 7 + j) for i in range(10) for j in range(10)])
    got, _ = oracle.cluster(hits, 20, 20, U64MAX, lib=lib)
    assert (got == np.arange(100)).all()
    # every corner and edge neighbourhood is clipped, not wrapped
    w, hh = 9, 7
    pts = [(0, 0), (w - 1, 0), (0, hh - 1), (w - 1, hh - 1), (w - 1, 2), (0, 3)]
    hits = make_hits([(x, y, 0) for x, y in pts])
    got, _ = oracle.cluster(hits, w, hh, U64MAX, lib=lib)
    assert (got == np.arange(len(pts))).all()


def pin_metamorphic(lib, seed=17):
    """Permuting the input, shifting every ToA and mirroring the sensor keep
    the partition (labels are re-minimised after a permutation)."""
    for c in range(30):
        rng = np.random.default_rng([seed, c])
        w, hh = 12, 10
        hits = hitgen.uniform_hits(int(rng.integers(1, 300)), [seed, c, 1], w, hh, 400)
        dt = int(rng.integers(0, 50))
        base, _ = oracle.cluster(hits, w, hh, dt, lib=lib)
        perm = rng.permutation(hits.size)
        got, _ = oracle.cluster(hits[perm], w, hh, dt, lib=lib)
        inv = np.argsort(perm)
        assert (canonical(perm[got][inv]) == base).all()
        sh = hits.copy()
        sh["toa"] += np.uint64(int(rng.integers(1, 1 << 50)))
        assert (oracle.cluster(sh, w, hh, dt, lib=lib)[0] == base).all()
        mx = hits.copy(); mx["x"] = w - 1 - mx["x"]
        assert (oracle.cluster(mx, w, hh, dt, lib=lib)[0] == base).all()
        my = hits.copy(); my["y"] = hh - 1 - my["y"]
        assert (oracle.cluster(my, w, hh, dt, lib=lib)[0] == base).all()


def pin_saturation(lib):
    """ToA near 0 with a large dt, ToA near 2^64-1 with dt = infinity."""
    hits = make_hits([(0, 0, 3), (1, 0, 1 << 40), (1, 1, 2)])
    got, _ = oracle.cluster(hits, 4, 4, 1 << 50, lib=lib)
    assert list(got) == [0, 0, 0]
    hits = make_hits([(0, 0, U64MAX), (1, 1, 0), (2, 2, U64MAX - 5)])
    got, _ = oracle.cluster(hits, 4, 4, U64MAX, lib=lib)
    assert list(got) == [0, 0, 0]
    got, _ = oracle.cluster(hits, 4, 4, 10, lib=lib)
    assert list(got) == [0, 1, 2]
    hits = make_hits([(0, 0, U64MAX - 5), (1, 1, U64MAX - 1), (5, 5, U64MAX)])
    got, _ = oracle.cluster(hits, 8, 8, 100, lib=lib)
    assert list(got) == [0, 0, 2]


def pin_features(lib, seed=19):
    rng = np.random.default_rng(seed)
    for c in range(40):
        w, hh = 30, 20
        hits = hitgen.uniform_hits(int(rng.integers(1, 400)), [seed, c], w, hh, 500)
        hits["tot"] = rng.integers(0, 3 if c % 4 == 0 else 65536, hits.size)
        dt = int(rng.integers(0, 60))
        lab, f = oracle.cluster(hits, w, hh, dt, lib=lib)
        assert features_equal(f, features_from_labels(hits, lab)), c
    # equal ToT: centroid is the arithmetic mean of the pixel coordinates
    hits = make_hits([(1, 1, 0, 9), (2, 1, 0, 9), (2, 2, 0, 9), (3, 3, 0, 9)])
    _, f = oracle.cluster(hits, 8, 8, 0, lib=lib)
    assert f.size == 1 and f[0]["cx"] == 2.0 and f[0]["cy"] == 7.0 / 4.0


def pin_blob_workload_invariants(lib):
    """The full 100k-hit blob workload: the independent window-scan partition
    and invariant checker agree, and the features recompute exactly."""
    hits, p = hitgen.blobs_100k()
    lab, f = oracle.cluster(hits, p["width"], p["height"], p["dt"], lib=lib)
    assert (lab == partition_of(hits, p["dt"])).all()
    check_invariants(hits, lab, p["dt"])
    assert features_equal(f, features_from_labels(hits, lab))


PINS = [pin_golden, pin_bruteforce, pin_image_labelling, pin_closed_forms, pin_metamorphic,
        pin_saturation, pin_features, pin_blob_workload_invariants]
