"""The multi-lane CPU baseline (the paper's CPU method: temporal splitting,
per-window sweeps, border merge cascade) gives the oracle's labels for any
number of lanes and any window length, including windows shorter than the
clusters (merges chained over many borders)."""
import numpy as np
import pytest

import cpu_lanes
import hitgen
import oracle


@pytest.mark.parametrize("lanes,window", [(1, 10 ** 12), (3, 40_000), (8, 2_000), (5, 128), (2, 64), (4, 1)])
def test_lanes_equal_oracle(lanes, window):
    hits, p = hitgen.mixed_10m(n=150_000, seed=7)
    want, _ = oracle.cluster(hits, 256, 256, p["dt"], features=False)
    got, k = cpu_lanes.cluster(hits, 256, 256, p["dt"], lanes, window)
    assert np.array_equal(got, want)
    assert k == np.unique(want).size


def test_lanes_special_cases():
    for hits, w, h, dt in [
        (hitgen.uniform_hits(5000, 8, width=8, height=8, toa_hi=2000), 8, 8, 3),
        (hitgen.uniform_hits(3000, 9, width=16, height=16, toa_hi=10 ** 6), 16, 16, (1 << 64) - 1),
        (hitgen.uniform_hits(3000, 10, width=16, height=16, toa_hi=400), 16, 16, 0),
        (hitgen.blobs_100k(n=20_000, seed=11)[0], 256, 256, 128),
    ]:
        want, _ = oracle.cluster(hits, w, h, dt, features=False)
        for lanes, window in ((1, 50), (6, 500), (16, 7)):
            got, _ = cpu_lanes.cluster(hits, w, h, dt, lanes, window)
            assert np.array_equal(got, want)
    got, k = cpu_lanes.cluster(np.empty(0, dtype=hitgen.HIT_DTYPE), 4, 4, 1, 2, 10)
    assert k == 0 and got.size == 0
