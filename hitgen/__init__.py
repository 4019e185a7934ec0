"""Seeded synthetic Timepix hit streams.

This module only *generates inputs*: it contains none of the clustering
arithmetic.  Both the GPU library's tests/benchmark and the oracle consume what
it produces, so it depends on neither.

The paper's datasets (gamma from Am-241, 40 GeV/c pions, 385 GeV/c lead ions)
are not available; these generators stand in for them with the shapes the
paper's workloads have: small compact blobs, long straight tracks, and heavy
blobs of hundreds of hits, arriving as a zero-suppressed stream that is only
partly sorted by ToA (the paper's "t-ordered" input, Section 3.1).

Every stream is built the same way:
  * clusters are drawn one after another, each emitting its hits;
  * the stream is ordered by ToA (stable), then locally shuffled by a stable
    sort on ``i + U{0..D}``, which moves no hit more than D positions;
  * ToT is ``min(65535, floor(exp(4 + 0.8 Z) + 0.5))`` with Z standard normal.

Random numbers come from numpy's PCG64 generator seeded explicitly, so a
(seed, parameters) pair always yields the same stream.
"""
import numpy as np

HIT_DTYPE = np.dtype([("toa", "<u8"), ("x", "<u2"), ("y", "<u2"), ("tot", "<u2"), ("reserved", "<u2")])

TPX3_TICK_NS = 1.5625          # Timepix3 ToA LSB
TPX4_TICK_NS = 25.0 / 128.0    # 195.3125 ps, Timepix4 fine ToA LSB
BASE_SEED = 241211809000

# the eight king moves
_DX = np.array([-1, 0, 1, -1, 1, -1, 0, 1], dtype=np.int64)
_DY = np.array([-1, -1, -1, 0, 0, 1, 1, 1], dtype=np.int64)


def ns_to_ticks(ns, tick_ns):
    """Whole ticks in ``ns`` nanoseconds (floor)."""
    return int(np.floor(ns / tick_ns + 1e-9))


def _fold(v, lo, hi):
    """Reflect integer positions into [lo, hi]; keeps unit steps unit steps."""
    span = hi - lo
    if span <= 0:
        return np.full_like(v, lo)
    m = np.mod(v - lo, 2 * span)
    return lo + np.where(m <= span, m, 2 * span - m)


def _tot(rng, m):
    z = rng.standard_normal(m)
    return np.minimum(65535.0, np.floor(np.exp(4.0 + 0.8 * z) + 0.5)).astype(np.uint16)


def _segments(sizes):
    sizes = np.asarray(sizes, dtype=np.int64)
    starts = np.cumsum(sizes) - sizes
    seg = np.repeat(np.arange(sizes.size, dtype=np.int64), sizes)
    return starts, seg


def _walk_offsets(rng, sizes, radius=None):
    """Per-hit (dx, dy) of random walks over king moves, one walk per cluster.

    With ``radius`` the walk is reflected inside the square |dx|,|dy| <= radius.
    """
    total = int(np.sum(sizes))
    starts, seg = _segments(sizes)
    d = rng.integers(0, 8, total)
    sx = _DX[d]
    sy = _DY[d]
    sx[starts] = 0
    sy[starts] = 0
    cx = np.cumsum(sx)
    cy = np.cumsum(sy)
    ox = cx - cx[starts][seg]
    oy = cy - cy[starts][seg]
    if radius is not None:
        ox = _fold(ox, -radius, radius)
        oy = _fold(oy, -radius, radius)
    return ox, oy, seg


def _blobs(rng, sizes, width, height, t0, jitter, radius=None):
    """Random-walk blobs: hit k of a blob has toa = t0 + U{0..jitter}."""
    ox, oy, seg = _walk_offsets(rng, sizes, radius)
    nb = len(sizes)
    x0 = rng.integers(0, width, nb)
    y0 = rng.integers(0, height, nb)
    x = _fold(x0[seg] + ox, 0, width - 1)
    y = _fold(y0[seg] + oy, 0, height - 1)
    toa = t0[seg] + rng.integers(0, jitter + 1, seg.size).astype(np.uint64)
    return x, y, toa, seg


def _tracks(rng, lengths, width, height, t0, step_max):
    """Straight tracks rasterised along their major axis (8-connected),
    clipped to the sensor; ToA grows by U{0..step_max} per pixel."""
    lengths = np.asarray(lengths, dtype=np.int64)
    nt = lengths.size
    starts, seg = _segments(lengths)
    k = np.arange(seg.size, dtype=np.int64) - starts[seg]
    theta = rng.uniform(0.0, 2.0 * np.pi, nt)
    c, s = np.cos(theta), np.sin(theta)
    m = np.maximum(np.abs(c), np.abs(s))
    ux, uy = c / m, s / m                      # one of them is exactly +-1
    x0 = rng.integers(0, width, nt)
    y0 = rng.integers(0, height, nt)
    x = x0[seg] + np.rint(k * ux[seg]).astype(np.int64)
    y = y0[seg] + np.rint(k * uy[seg]).astype(np.int64)
    inc = rng.integers(0, step_max + 1, seg.size).astype(np.uint64)
    inc[starts] = 0
    cum = np.cumsum(inc)
    toa = t0[seg] + (cum - cum[starts][seg])
    keep = (x >= 0) & (x < width) & (y >= 0) & (y < height)
    return x[keep], y[keep], toa[keep], seg[keep]


def _assemble(rng, x, y, toa, n, disorder):
    """Truncate to n hits, order by ToA, then shuffle locally by <= disorder."""
    x, y, toa = x[:n], y[:n], toa[:n]
    hits = np.empty(x.size, dtype=HIT_DTYPE)
    hits["x"] = x
    hits["y"] = y
    hits["toa"] = toa
    hits["tot"] = _tot(rng, x.size)
    hits["reserved"] = 0
    hits = hits[np.argsort(hits["toa"], kind="stable")]
    if disorder > 0 and hits.size > 1:
        key = np.arange(hits.size, dtype=np.int64) + rng.integers(0, disorder + 1, hits.size)
        hits = hits[np.argsort(key, kind="stable")]
    return hits


def realised_disorder_ticks(hits):
    """max over i < j of toa_i - toa_j (0 if sorted): the paper's t."""
    t = hits["toa"].astype(np.uint64)
    if t.size < 2:
        return 0
    pm = np.maximum.accumulate(t)[:-1]
    d = pm.astype(np.int64) - t[1:].astype(np.int64)
    return int(max(0, d.max()))


def blob_stream(n, seed, width=256, height=256, span_ticks=6_400_000, jitter=64,
                mean_size=6.0, size_cap=40, disorder=512):
    """Config-1 style stream: random-walk blobs, size min(cap, Geom(1/mean)),
    seed ToA uniform over ``span_ticks``, per-hit ToA seed + U{0..jitter}."""
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.empty(0, dtype=HIT_DTYPE)
    parts_x, parts_y, parts_t = [], [], []
    have = 0
    while have < n:
        nb = max(16, int((n - have) / mean_size * 1.1) + 16)
        sizes = np.minimum(size_cap, rng.geometric(1.0 / mean_size, nb))
        t0 = rng.integers(0, max(1, span_ticks), nb).astype(np.uint64)
        x, y, toa, _ = _blobs(rng, sizes, width, height, t0, jitter)
        parts_x.append(x); parts_y.append(y); parts_t.append(toa)
        have += x.size
    return _assemble(rng, np.concatenate(parts_x), np.concatenate(parts_y),
                     np.concatenate(parts_t), n, disorder)


def mixed_stream(n, seed, width=256, height=256, span_ticks=640_000_000, disorder=4096,
                 blob_jitter=64, track_step=32, heavy_radius=15):
    """Config-2 style stream: 70 % small blobs (size U{1..10}), 25 % straight
    tracks (length U{20..200}, ToA +U{0..track_step} per pixel), 5 % heavy
    blobs (U{200..500} hits reflected inside |dx|,|dy| <= heavy_radius)."""
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.empty(0, dtype=HIT_DTYPE)
    parts = []
    have = 0
    while have < n:
        nc = max(64, int((n - have) / 48.0 * 1.1) + 64)
        kind = rng.choice(3, size=nc, p=[0.70, 0.25, 0.05])
        # cluster order is interleaved only through their seed ToA, so each
        # kind can be generated as a block
        t0 = rng.integers(0, max(1, span_ticks), nc).astype(np.uint64)
        nsmall, ntrack, nheavy = (int((kind == k).sum()) for k in range(3))
        xs, ys, ts = [], [], []
        if nsmall:
            x, y, t, _ = _blobs(rng, rng.integers(1, 11, nsmall), width, height,
                                t0[kind == 0], blob_jitter)
            xs.append(x); ys.append(y); ts.append(t)
        if ntrack:
            x, y, t, _ = _tracks(rng, rng.integers(20, 201, ntrack), width, height,
                                 t0[kind == 1], track_step)
            xs.append(x); ys.append(y); ts.append(t)
        if nheavy:
            x, y, t, _ = _blobs(rng, rng.integers(200, 501, nheavy), width, height,
                                t0[kind == 2], blob_jitter, radius=heavy_radius)
            xs.append(x); ys.append(y); ts.append(t)
        x, y, t = np.concatenate(xs), np.concatenate(ys), np.concatenate(ts)
        # shuffle the cluster blocks' hits so truncation does not favour a kind
        p = rng.permutation(x.size)
        parts.append((x[p], y[p], t[p]))
        have += x.size
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    t = np.concatenate([p[2] for p in parts])
    return _assemble(rng, x, y, t, n, disorder)


def shower_stream(n, seed, width=256, height=256, span_ticks=None, disorder=4096,
                  shower_hits=(1500, 6000), shower_share=0.3, radius=40, jitter=64):
    """The mixed stream (``mixed_stream``) with dense showers added: about
    ``shower_share`` of the n hits arrive in showers of U{shower_hits} hits
    each within ``jitter`` ticks, a random walk reflected inside the square
    |dx|,|dy| <= radius around a uniform origin.  Every later hit of a shower
    has hundreds to thousands of earlier hits within dt before it."""
    rng = np.random.default_rng(seed)
    if n == 0:
        return np.empty(0, dtype=HIT_DTYPE)
    if span_ticks is None:
        span_ticks = int(round(n / 10e6 * 1e9 / TPX3_TICK_NS))
    lo, hi = shower_hits
    sizes = []
    want = int(n * shower_share)
    while sum(sizes) < want:
        sizes.append(int(rng.integers(lo, hi + 1)))
    sizes = np.array(sizes, dtype=np.int64)
    t0 = rng.integers(0, max(1, span_ticks), sizes.size).astype(np.uint64)
    sx, sy, st, _ = _blobs(rng, sizes, width, height, t0, jitter, radius=radius)
    base = mixed_stream(max(0, n - int(sizes.sum())), int(rng.integers(1 << 62)), width, height,
                        span_ticks=span_ticks, disorder=0, blob_jitter=jitter,
                        track_step=max(1, jitter // 2), heavy_radius=15)
    x = np.concatenate([base["x"].astype(np.int64), sx])
    y = np.concatenate([base["y"].astype(np.int64), sy])
    t = np.concatenate([base["toa"], st])
    p = rng.permutation(x.size)
    return _assemble(rng, x[p], y[p], t[p], n, disorder)


# ---------------------------------------------------------------------------
# the named workloads


def blobs_100k(n=100_000, seed=BASE_SEED + 1):
    """Single Timepix3 256x256 sensor, 100k hits of random-walk blobs
    (size min(40, Geom(mean 6))), seeds over 10 ms, ToA jitter 100 ns,
    displacement <= 512, dt = 200 ns.  Returns (hits, params)."""
    hits = blob_stream(n, seed, 256, 256, span_ticks=ns_to_ticks(10e6, TPX3_TICK_NS),
                       jitter=ns_to_ticks(100, TPX3_TICK_NS), mean_size=6.0, size_cap=40,
                       disorder=512)
    return hits, dict(width=256, height=256, dt=ns_to_ticks(200, TPX3_TICK_NS), disorder=512)


def mixed_10m(n=10_000_000, seed=BASE_SEED + 2, span_ticks=None):
    """Single 256x256 sensor, ~10 Mhit/s mixed blobs/tracks/heavy blobs over
    about 1 s, displacement <= 4096, dt = 200 ns.  Returns (hits, params)."""
    if span_ticks is None:
        span_ticks = int(round(n / 10e6 * 1e9 / TPX3_TICK_NS))  # keep 10 Mhit/s
    hits = mixed_stream(n, seed, 256, 256, span_ticks=span_ticks, disorder=4096,
                        blob_jitter=ns_to_ticks(100, TPX3_TICK_NS),
                        track_step=ns_to_ticks(50, TPX3_TICK_NS), heavy_radius=15)
    return hits, dict(width=256, height=256, dt=ns_to_ticks(200, TPX3_TICK_NS), disorder=4096)


def batch64_sizes(seed=BASE_SEED + 3, chunks=64, lo=1e3, hi=2e6, target=30e6, tol=0.10):
    """Log-uniform chunk sizes; the first sub-seed whose total lies within
    target +- tol is used (the plain log-uniform mean is ~16.8 M)."""
    for sub in range(100000):
        rng = np.random.default_rng([seed, sub])
        sizes = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), chunks))).astype(np.int64)
        if abs(sizes.sum() - target) <= tol * target:
            return sizes, sub
    raise RuntimeError("no sub-seed found")


def batch_64_chunks(seed=BASE_SEED + 3, scale=1.0):
    """64 chunks from 4 detectors, each a blob stream with its own dt in
    {100, 200, 500} ns; ``scale`` shrinks every chunk (tests).  Returns
    (list of hit arrays, list of dt ticks, detector ids)."""
    sizes, sub = batch64_sizes(seed)
    rng = np.random.default_rng([seed, sub, 1])
    dts_ns = rng.choice([100, 200, 500], size=sizes.size)
    chunks, dts = [], []
    for c, nc in enumerate(sizes):
        nc = max(1, int(nc * scale))
        span = int(round(nc / 10e6 * 1e9 / TPX3_TICK_NS))
        h = blob_stream(nc, [seed, sub, 2, c], 256, 256, span_ticks=span,
                        jitter=ns_to_ticks(100, TPX3_TICK_NS), disorder=512)
        chunks.append(h)
        dts.append(ns_to_ticks(float(dts_ns[c]), TPX3_TICK_NS))
    return chunks, dts, [c % 4 for c in range(sizes.size)]


def timepix4_200m(n=200_000_000, seed=BASE_SEED + 4):
    """Timepix4-shaped 448x512 sensor at 300 Mhit/s: random-walk blobs of
    size min(60, Geom(mean 9)), ToA ticks of 195.3125 ps, displacement <= 16384,
    dt = 200 ns = 1024 ticks.  Returns (hits, params)."""
    span = int(round(n / 300e6 * 1e9 / TPX4_TICK_NS))
    hits = blob_stream(n, seed, 448, 512, span_ticks=span,
                       jitter=ns_to_ticks(100, TPX4_TICK_NS), mean_size=9.0, size_cap=60,
                       disorder=16384)
    return hits, dict(width=448, height=512, dt=ns_to_ticks(200, TPX4_TICK_NS), disorder=16384)


def uniform_hits(n, seed, width=8, height=8, toa_hi=64, disorder=None):
    """Hits uniform over a small box and time range (dense, many collisions)."""
    rng = np.random.default_rng(seed)
    hits = np.empty(n, dtype=HIT_DTYPE)
    hits["x"] = rng.integers(0, width, n)
    hits["y"] = rng.integers(0, height, n)
    hits["toa"] = rng.integers(0, max(1, toa_hi), n).astype(np.uint64)
    hits["tot"] = rng.integers(0, 100, n)
    hits["reserved"] = 0
    if disorder is not None:
        hits = hits[np.argsort(hits["toa"], kind="stable")]
        key = np.arange(n) + rng.integers(0, disorder + 1, n)
        hits = hits[np.argsort(key, kind="stable")]
    return hits


# ---------------------------------------------------------------------------
# the Timepix4-shaped stream, generated window by window


TPX4_PARAMS = dict(width=448, height=512, dt=ns_to_ticks(200, TPX4_TICK_NS), disorder=16384)


def _tpx4_window(seed, w, hits_per_window, span_ticks):
    """Raw (unsorted) hits of window w: blobs of min(60, Geom(1/9)) hits drawn
    until the window holds at least hits_per_window hits, seeds uniform over
    [w * span, (w + 1) * span), per-hit ToA seed + U{0..100 ns}, ToT as
    everywhere."""
    rng = np.random.default_rng([seed, w])
    nb = int(hits_per_window / 9.0 * 1.1) + 64
    while True:
        sizes = np.minimum(60, rng.geometric(1.0 / 9.0, nb))
        c = np.cumsum(sizes)
        if c[-1] >= hits_per_window:
            sizes = sizes[: int(np.searchsorted(c, hits_per_window)) + 1]
            break
        nb *= 2
    t0 = (np.uint64(w * span_ticks) +
          rng.integers(0, span_ticks, sizes.size).astype(np.uint64))
    x, y, toa, _ = _blobs(rng, sizes, 448, 512, t0, ns_to_ticks(100, TPX4_TICK_NS))
    out = np.empty(x.size, dtype=HIT_DTYPE)
    out["x"], out["y"], out["toa"] = x, y, toa
    out["tot"] = _tot(rng, x.size)
    out["reserved"] = 0
    return out


def timepix4_stream(n=200_000_000, seed=BASE_SEED + 4, window=1 << 20, workers=8):
    """The Timepix4-shaped stream (448x512 sensor, 300 Mhit/s, 195.3125 ps
    ticks, blobs of min(60, Geom(mean 9)) hits, displacement <= 16384) as a
    generator of consecutive pieces, without ever holding the whole stream.

    Window w draws clusters whose seed ToAs lie in [w * S, (w + 1) * S), S
    being the time 300 Mhit/s needs for ``window`` hits; the stream stops after
    n hits, at a ToA (the earliest hits of the last window), so the rate
    holds to the end.  The ToA sort is
    done window by window: hits below the next window's start are final,
    later ones wait for the next window, which makes the result the stable
    ToA order of the whole stream.  The local shuffle (stable sort on
    i + U{0..D}) likewise: once positions below P are all known, every key
    below P is final.  Windows are generated in parallel threads."""
    from concurrent.futures import ThreadPoolExecutor
    D = TPX4_PARAMS["disorder"]
    span = int(round(window / 300e6 * 1e9 / TPX4_TICK_NS))
    left = n
    carry = np.empty(0, dtype=HIT_DTYPE)
    pend_key = np.empty(0, dtype=np.int64)
    pend_hits = np.empty(0, dtype=HIT_DTYPE)
    pos = 0  # sorted positions handed out so far
    ex = ThreadPoolExecutor(max_workers=max(1, workers))
    futs = {}
    w = 0
    try:
        while True:
            for k in range(w, w + 2 * max(1, workers)):
                if k not in futs:
                    futs[k] = ex.submit(_tpx4_window, seed, k, window, span)
            if left > 0:
                raw = futs.pop(w).result()
                take = min(left, raw.size)
                left -= raw.size
            else:
                futs.pop(w).cancel()
                raw = np.empty(0, dtype=HIT_DTYPE)
                take = 0
            pool = np.concatenate([carry, raw])
            pool = pool[np.argsort(pool["toa"], kind="stable")]
            last = left <= 0
            if last:
                # the stream stops at a ToA: the earliest hits up to n in all
                done, carry = pool[: carry.size + take], pool[:0]
            else:
                cut = int(np.searchsorted(pool["toa"], np.uint64((w + 1) * span), side="left"))
                done, carry = pool[:cut], pool[cut:]
            # local shuffle of the newly final sorted positions
            rng = np.random.default_rng([seed, w, 7])
            keys = np.arange(pos, pos + done.size, dtype=np.int64) + rng.integers(0, D + 1, done.size)
            pos += done.size
            pend_key = np.concatenate([pend_key, keys])
            pend_hits = np.concatenate([pend_hits, done])
            order = np.argsort(pend_key, kind="stable")  # pending items are in position order
            if last:
                yield pend_hits[order]
                return
            nfin = int(np.count_nonzero(pend_key < pos))  # keys below pos lead `order`
            out = pend_hits[order[:nfin]]
            keep = np.ones(pend_key.size, dtype=bool)  # the rest stays in position order
            keep[order[:nfin]] = False
            pend_key, pend_hits = pend_key[keep], pend_hits[keep]
            if out.size:
                yield out
            w += 1
    finally:
        for f in futs.values():
            f.cancel()
        ex.shutdown(wait=False, cancel_futures=True)


def pieces(gen, size):
    """Re-cut a generator of hit arrays into consecutive arrays of ``size``
    hits (the last one shorter)."""
    buf, have = [], 0
    for a in gen:
        buf.append(a)
        have += a.size
        while have >= size:
            cat = np.concatenate(buf)
            yield cat[:size]
            buf, have = [cat[size:]], have - size
    if have:
        yield np.concatenate(buf)
