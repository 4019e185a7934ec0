"""CPU emulation of the tiled ToA ordering (sort tiles of T hits, rank every
element against the m neighbour tiles on each side): whenever the check on
the tile minimum/maximum keys passes, the ranks are exactly the positions in
(toa, index) order, and a displacement of at most m*T/2 always passes it --
also when the last tile is short.  The check: tile j's maximum lies below
the minimum of tile j+m+1, and the tile minima ascend from tile m+1 on
(together: every tile m+1 or more places after j lies wholly above j).  The
first m+1 tiles may be in any order among themselves, as in a stream's
buffer whose open hits precede the new chunk.  Also the merge-path form of
the neighbour counts (equal shares of the merged sequence per thread)."""
import numpy as np
import pytest

import hitgen


def tile_ranks(toa, T, m):
    """Returns (ranks or None if the check fails)."""
    n = toa.size
    idx = np.arange(n)
    nt = (n + T - 1) // T
    tiles = []
    for j in range(nt):
        a, b = j * T, min(n, (j + 1) * T)
        o = np.lexsort((idx[a:b], toa[a:b]))
        keys = list(zip(toa[a:b][o].tolist(), (a + o).tolist()))
        tiles.append(keys)
    for j in range(nt):
        if j + 1 < nt and j >= m + 1 and tiles[j + 1][0] < tiles[j][0]:
            return None
        if j + m + 1 < nt and not tiles[j][-1] < tiles[j + m + 1][0]:
            return None
    ranks = np.empty(n, dtype=np.int64)
    for j in range(nt):
        lo_t, hi_t = max(0, j - m), min(nt - 1, j + m)
        for r, key in enumerate(tiles[j]):
            rank = lo_t * T + r
            for i in range(lo_t, hi_t + 1):
                if i != j:
                    rank += sum(1 for k in tiles[i] if k < key)
            ranks[key[1]] = rank
    return ranks


def true_ranks(toa):
    order = np.lexsort((np.arange(toa.size), toa))
    r = np.empty(toa.size, dtype=np.int64)
    r[order] = np.arange(toa.size)
    return r


@pytest.mark.parametrize("seed", range(12))
def test_ranks_exact_when_check_passes(seed):
    rng = np.random.default_rng(seed)
    T = int(rng.choice([8, 16, 32]))
    n = int(rng.integers(1, 6 * T))
    D = int(rng.integers(0, 2 * T))
    m = max(1, -(-2 * D // T))
    toa = np.sort(rng.integers(0, 3 * n, n)).astype(np.int64)
    key = np.arange(n) + rng.integers(0, D + 1, n)
    toa = toa[np.argsort(key, kind="stable")]
    r = tile_ranks(toa, T, m)
    if D <= m * T // 2:
        assert r is not None, "displacement within the bound must pass the check"
    if r is not None:
        assert np.array_equal(r, true_ranks(toa))


@pytest.mark.parametrize("seed", range(10))
def test_ranks_exact_with_unordered_prefix(seed):
    """A prefix of hits whose ToAs interleave with the following ones (a
    stream's open hits before a chunk), then a locally shuffled tail: the
    relaxed check passes with m covering the prefix, and the ranks are exact;
    any other input that passes is exact too."""
    rng = np.random.default_rng(500 + seed)
    T = int(rng.choice([8, 16]))
    pre = int(rng.integers(1, 3 * T))
    tail = int(rng.integers(T, 8 * T))
    D = int(rng.integers(0, T))
    toa_tail = np.sort(rng.integers(0, 4 * tail, tail)).astype(np.int64)
    toa_tail = toa_tail[np.argsort(np.arange(tail) + rng.integers(0, D + 1, tail), kind="stable")]
    # the prefix lies among the tail's first hits in ToA
    toa_pre = rng.integers(0, max(1, int(toa_tail[: pre + 1].max())) + 1, pre).astype(np.int64)
    toa = np.concatenate([toa_pre, toa_tail])
    m = max(1, -(-2 * (D + pre) // T))
    r = tile_ranks(toa, T, m)
    assert r is not None
    assert np.array_equal(r, true_ranks(toa))


@pytest.mark.parametrize("seed", range(6))
def test_any_input_passing_the_check_is_exact(seed):
    rng = np.random.default_rng(900 + seed)
    passed = 0
    for _ in range(300):
        T = int(rng.choice([4, 8]))
        n = int(rng.integers(1, 10 * T))
        m = int(rng.integers(1, 4))
        kind = int(rng.integers(0, 3))
        if kind == 0:  # random
            toa = rng.integers(0, 3 * n, n).astype(np.int64)
        elif kind == 1:  # scrambled head, sorted rest
            toa = np.sort(rng.integers(0, 3 * n, n)).astype(np.int64)
            h = int(rng.integers(0, n + 1))
            toa[:h] = rng.permutation(toa[:h])
        else:  # sorted with random swaps anywhere
            toa = np.sort(rng.integers(0, 3 * n, n)).astype(np.int64)
            for _ in range(int(rng.integers(0, 4))):
                a, b = rng.integers(0, n, 2)
                toa[a], toa[b] = toa[b], toa[a]
        r = tile_ranks(toa, T, m)
        if r is not None:
            passed += 1
            assert np.array_equal(r, true_ranks(toa)), (T, m, toa.tolist())
    assert passed > 50


def test_short_last_tile_passes():
    # T = 16, 51 hits: the last tile holds 3.  Swapping positions 40 and 50
    # (displacement 10) leaves the last tile's maximum below tile 2's; tile
    # minima still ascend and the gap rule holds, and the ranks are exact.
    T, D = 16, 10
    toa = np.arange(3 * T + 3, dtype=np.int64)
    toa[40], toa[50] = 50, 40
    m = max(1, -(-2 * D // T))
    r = tile_ranks(toa, T, m)
    assert r is not None
    assert np.array_equal(r, true_ranks(toa))


def test_blob_stream_ranks():
    h = hitgen.blob_stream(700, 3, span_ticks=700 * 64, disorder=24)
    toa = h["toa"].astype(np.int64)
    for T in (64, 128):
        m = max(1, -(-2 * 24 // T))
        r = tile_ranks(toa, T, m)
        assert r is not None
        assert np.array_equal(r, true_ranks(toa))


def merge_path_counts(A, B, earlier, threads):
    """The tile rank's neighbour counts: for every key of the sorted tile A,
    how many keys of the sorted neighbour B go before it (B <= A for an
    earlier neighbour, whose indices are smaller; B < A for a later one),
    each of `threads` threads merging an equal share of the merged sequence
    after one binary search for where its share starts."""
    na, nb = len(A), len(B)
    below = [None] * na

    def b_first(bi, ai):
        return B[bi] <= A[ai] if earlier else B[bi] < A[ai]

    total = na + nb
    per = -(-total // threads)
    for t in range(threads):
        d0 = min(t * per, total)
        d1 = min(d0 + per, total)
        lo, hi = max(d0 - nb, 0), min(d0, na)
        while lo < hi:
            mid = (lo + hi) >> 1
            if not b_first(d0 - mid - 1, mid):
                lo = mid + 1
            else:
                hi = mid
        ai, bi = lo, d0 - lo
        for _ in range(d0, d1):
            if bi < nb and (ai == na or b_first(bi, ai)):
                bi += 1
            else:
                assert below[ai] is None, "an element placed twice"
                below[ai] = bi
                ai += 1
    return below


@pytest.mark.parametrize("seed", range(8))
def test_merge_path_counts(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(200):
        na, nb = int(rng.integers(1, 70)), int(rng.integers(1, 70))
        threads = int(rng.integers(1, 24))
        span = int(rng.integers(1, 50))  # small spans: many equal keys
        off = int(rng.integers(-span, span + 1))  # partial, full or no overlap
        A = sorted(rng.integers(0, span, na).tolist())
        B = sorted((rng.integers(0, span, nb) + off).tolist())
        for earlier in (True, False):
            want = [sum(1 for b in B if (b <= a if earlier else b < a)) for a in A]
            assert merge_path_counts(A, B, earlier, threads) == want
