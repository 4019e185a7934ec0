"""The neighbour rules the link kernels rely on, checked on the CPU.

The kernel processes the ToA-sorted hits in tiles; every tile hit joins, at
each pixel of its 3x3 neighbourhood, only the LATEST earlier hit there (if it
is within dt), looking back no further than the tile's halo (the hits within
dt before the tile's first hit).  This is a restatement of the paper's sweep
with a per-pixel "last hit" matrix (Section 4.1) cut into independent tiles.
This test emulates exactly that rule in plain Python and compares the result
with the oracle, at tile sizes small enough that many clusters cross tiles.
The pixel-index kernel relaxes it further -- ANY earlier hit within dt at
each neighbour pixel -- which gives the same clusters (tested below with
several choices, and a counterexample showing that later hits may not be
offered).
"""
import numpy as np
import pytest

import hitgen
import oracle
from refs import canonical


def tiled_rule_labels(hits, width, height, dt, tile=64):
    n = hits.size
    order = np.lexsort((np.arange(n), hits["toa"]))
    toa = hits["toa"][order].astype(np.uint64)
    x = hits["x"][order].astype(np.int64)
    y = hits["y"][order].astype(np.int64)
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for p0 in range(0, n, tile):
        p1 = min(n, p0 + tile)
        lo = int(toa[p0]) - dt if int(toa[p0]) > dt else 0
        h0 = int(np.searchsorted(toa[:p0], np.uint64(lo), side="left"))
        last = {}
        for i in range(h0, p1):
            if i >= p0:
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        qx, qy = x[i] + dx, y[i] + dy
                        if 0 <= qx < width and 0 <= qy < height:
                            a = last.get((qx, qy))
                            if a is not None and int(toa[i]) - int(toa[a]) <= dt:
                                ra, rb = find(a), find(i)
                                if ra != rb:
                                    parent[max(ra, rb)] = min(ra, rb)
            last[(x[i], y[i])] = i
    lab = np.empty(n, dtype=np.int64)
    lab[order] = [find(i) for i in range(n)]
    return canonical(lab)


@pytest.mark.parametrize("case", ["blobs", "mixed", "dense"])
def test_tiled_latest_hit_rule_matches_oracle(case):
    if case == "blobs":
        hits, p = hitgen.blobs_100k(n=20_000, seed=31)
        w, h, dt = 256, 256, p["dt"]
    elif case == "mixed":
        hits, p = hitgen.mixed_10m(n=30_000, seed=32)
        w, h, dt = 256, 256, p["dt"]
    else:
        hits = hitgen.uniform_hits(5_000, 33, 12, 12, 20_000, disorder=40)
        w, h, dt = 12, 12, 25
    want, _ = oracle.cluster(hits, w, h, dt)
    got = tiled_rule_labels(hits, w, h, dt, tile=64)
    assert (got == want).all()


def tiled_any_rule_labels(hits, width, height, dt, tile, choose, earlier_only=True):
    """The pixel index's form of the rule: every tile hit joins, at each pixel
    of its 3x3 neighbourhood, ONE earlier hit of the tile or its halo that is
    within dt, picked by ``choose(candidates, time_distances)`` from all of
    them (not necessarily the latest).  earlier_only=False also offers the
    later hits within dt (a rule that is NOT exact)."""
    n = hits.size
    order = np.lexsort((np.arange(n), hits["toa"]))
    toa = hits["toa"][order].astype(np.int64)
    x = hits["x"][order].astype(np.int64)
    y = hits["y"][order].astype(np.int64)
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for p0 in range(0, n, tile):
        p1 = min(n, p0 + tile)
        h0 = int(np.searchsorted(toa[:p0], max(int(toa[p0]) - dt, 0), side="left"))
        at = {}
        for j in range(h0, p1):
            at.setdefault((x[j], y[j]), []).append(j)
        for i in range(p0, p1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ok = [j for j in at.get((x[i] + dx, y[i] + dy), ())
                          if (j < i or (not earlier_only and j != i)) and abs(toa[i] - toa[j]) <= dt]
                    if ok:
                        ra, rb = find(choose(ok, [abs(toa[i] - toa[j]) for j in ok])), find(i)
                        if ra != rb:
                            parent[max(ra, rb)] = min(ra, rb)
    lab = np.empty(n, dtype=np.int64)
    lab[order] = [find(i) for i in range(n)]
    return canonical(lab)


def _earliest(ok, dist):
    return min(ok)


def _farthest(ok, dist):
    return ok[int(np.argmax(dist))]


@pytest.mark.parametrize("case", ["mixed", "dense"])
@pytest.mark.parametrize("pick", ["earliest", "farthest", "random"])
def test_tiled_any_earlier_hit_rule_matches_oracle(case, pick):
    if case == "mixed":
        hits, p = hitgen.mixed_10m(n=20_000, seed=34)
        w, h, dt = 256, 256, p["dt"]
    else:
        hits = hitgen.uniform_hits(4_000, 35, 10, 10, 12_000, disorder=40)
        w, h, dt = 10, 10, 25
    rng = np.random.default_rng(36)
    choose = {"earliest": _earliest, "farthest": _farthest,
              "random": lambda ok, dist: ok[int(rng.integers(len(ok)))]}[pick]
    want, _ = oracle.cluster(hits, w, h, dt)
    got = tiled_any_rule_labels(hits, w, h, dt, 64, choose)
    assert (got == want).all()


def test_any_hit_rule_must_look_back_only():
    # a (P, t=0) and b (Q, t=50) are neighbours within dt = 60, so the oracle
    # keeps j (Q, -60), a, b and a2 (P, 110) in one cluster.  Offered later
    # hits too, a may pick j and b may pick a2 and the cluster splits; with
    # earlier hits only, b must pick a.
    hits = _rows([(0, 0, 0), (1, 0, -60), (1, 0, 50), (0, 0, 110)], base=1000)
    want, _ = oracle.cluster(hits, 4, 4, 60)
    assert len(set(want.tolist())) == 1
    assert (tiled_any_rule_labels(hits, 4, 4, 60, 64, _farthest) == want).all()
    split = tiled_any_rule_labels(hits, 4, 4, 60, 64, _farthest, earlier_only=False)
    assert len(set(split.tolist())) == 2


def _rows(rows, base):
    h = np.zeros(len(rows), dtype=oracle.HIT_DTYPE)
    for k, (xx, yy, t) in enumerate(rows):
        h[k]["x"], h[k]["y"], h[k]["toa"], h[k]["tot"] = xx, yy, base + t, 1
    return h


# ---- the time-window form of the same rule (the default link kernel)
GUARD, MASK = np.uint32(0x40004000), np.uint32(0xFFFCFFFC)


def swar_adjacent(gx, gy, ix, iy):
    """The kernel's two-lane test: returns (adjacent, direction 0..8) for
    earlier hit (gx, gy) and hit (ix, iy), coordinates below 2^14."""
    g = (np.uint32(gy) << np.uint32(16) | np.uint32(gx)) | GUARD
    c = np.uint32((int(iy) << 16 | int(ix)) - 0x00010001 & 0xFFFFFFFF)
    r = np.uint32((int(g) - int(c)) & 0xFFFFFFFF)
    if (r & MASK) != GUARD:
        return False, -1
    ax, ay = int(r & 3), int((r >> 16) & 3)
    if ax == 3 or ay == 3:
        return False, -1
    return True, ay * 3 + ax


def test_swar_adjacency_predicate():
    rng = np.random.default_rng(5)
    pts = [(0, 0), (16383, 16383), (0, 16383), (16383, 0), (1, 1)] + \
          [tuple(rng.integers(0, 16384, 2)) for _ in range(200)]
    for ix, iy in pts:
        for dy in range(-3, 4):
            for dx in range(-3, 4):
                gx, gy = ix + dx, iy + dy
                if not (0 <= gx < 16384 and 0 <= gy < 16384):
                    continue
                adj, d = swar_adjacent(gx, gy, ix, iy)
                assert adj == (abs(dx) <= 1 and abs(dy) <= 1), (ix, iy, dx, dy)
                if adj:
                    assert d == (dy + 1) * 3 + (dx + 1)
    # far apart in both lanes, including differences that would borrow
    for _ in range(2000):
        ix, iy, gx, gy = rng.integers(0, 16384, 4)
        adj, _ = swar_adjacent(gx, gy, ix, iy)
        assert adj == (abs(int(gx) - int(ix)) <= 1 and abs(int(gy) - int(iy)) <= 1)


def window_rule_labels(hits, width, height, dt, tile=64):
    n = hits.size
    order = np.lexsort((np.arange(n), hits["toa"]))
    toa = hits["toa"][order].astype(np.uint64)
    x = hits["x"][order].astype(np.int64)
    y = hits["y"][order].astype(np.int64)
    g_all = ((y << 16) | x).astype(np.uint64) | np.uint64(0x40004000)
    parent = list(range(n))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for p0 in range(0, n, tile):
        p1 = min(n, p0 + tile)
        lo0 = int(toa[p0]) - dt if int(toa[p0]) > dt else 0
        h0 = int(np.searchsorted(toa[:p0], np.uint64(lo0), side="left"))
        for i in range(p0, p1):
            lo_t = int(toa[i]) - dt if int(toa[i]) > dt else 0
            lo = h0 + int(np.searchsorted(toa[h0:i], np.uint64(lo_t), side="left"))
            if lo >= i:
                continue
            c = (int((y[i] << 16) | x[i]) - 0x00010001) & 0xFFFFFFFF
            r = ((g_all[lo:i] - np.uint64(c)) & np.uint64(0xFFFFFFFF))[::-1]  # j = i-1 down to lo
            ok = (r & np.uint64(0xFFFCFFFC)) == np.uint64(0x40004000)
            ax, ay = r & np.uint64(3), (r >> np.uint64(16)) & np.uint64(3)
            ok &= (ax != 3) & (ay != 3)
            seen = set()
            for k in np.nonzero(ok)[0]:
                d = int(ay[k]) * 3 + int(ax[k])
                if d in seen:
                    continue
                seen.add(d)
                j = i - 1 - int(k)
                ra, rb = find(j), find(i)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    lab = np.empty(n, dtype=np.int64)
    lab[order] = [find(i) for i in range(n)]
    return canonical(lab)


@pytest.mark.parametrize("case", ["blobs", "mixed", "dense"])
def test_window_rule_matches_oracle(case):
    if case == "blobs":
        hits, p = hitgen.blobs_100k(n=20_000, seed=41)
        w, h, dt = 256, 256, p["dt"]
    elif case == "mixed":
        hits, p = hitgen.mixed_10m(n=30_000, seed=42)
        w, h, dt = 256, 256, p["dt"]
    else:
        hits = hitgen.uniform_hits(5_000, 43, 12, 12, 20_000, disorder=40)
        w, h, dt = 12, 12, 25
    want, _ = oracle.cluster(hits, w, h, dt)
    got = window_rule_labels(hits, w, h, dt, tile=64)
    assert (got == want).all()
