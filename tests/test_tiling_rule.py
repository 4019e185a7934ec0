"""The neighbour rule the link kernel relies on, checked on the CPU.

The kernel processes the ToA-sorted hits in tiles; every tile hit joins, at
each pixel of its 3x3 neighbourhood, only the LATEST earlier hit there (if it
is within dt), looking back no further than the tile's halo (the hits within
dt before the tile's first hit).  This is a restatement of the paper's sweep
with a per-pixel "last hit" matrix (Section 4.1) cut into independent tiles.
This test emulates exactly that rule in plain Python and compares the result
with the oracle, at tile sizes small enough that many clusters cross tiles.
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
        hits, p = hitgen.config1(n=20_000, seed=31)
        w, h, dt = 256, 256, p["dt"]
    elif case == "mixed":
        hits, p = hitgen.config2(n=30_000, seed=32)
        w, h, dt = 256, 256, p["dt"]
    else:
        hits = hitgen.uniform_hits(5_000, 33, 12, 12, 20_000, disorder=40)
        w, h, dt = 12, 12, 25
    want, _ = oracle.cluster(hits, w, h, dt)
    got = tiled_rule_labels(hits, w, h, dt, tile=64)
    assert (got == want).all()
