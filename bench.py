"""Benchmark of the plain clustering path on one MI355X.

One step = one hc_cluster call over the whole workload (sort, neighbour
search + union-find, flatten, features, compaction), hits already resident in
HBM.  Workload: 256x256 Timepix3 sensor, 10M hits over ~1 s of mixed small
blobs, straight tracks and heavy blobs, locally shuffled by up to 4096
positions, dt = 200 ns (128 ticks of 1.5625 ns).  Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "clustered Mhits/s on 1 MI355X (batched/served vs plain) + p99 chunk latency"
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes of each kernel: what its contract must read once and
# write once, per hit and per cluster.  The whole path's figure is 20 B per
# hit (read the 16-byte hit, write the 4-byte label) + 64 B per cluster.
ALG_BYTES = {
    "tile_sort": (16 + 12, 0),   # hit record in; relative ToA + payload (index, ToT, pixel) out
    "tile_rank": (12 + 18, 0),   # relative ToA + payload in; sorted ToA, pixel, ToT, index out
    "link": (16 + 4, 0),         # sorted ToA, pixel, index in; parent out
    "flatten": (4 + 4, 0),       # parent in; label out
    "features": (22, 64),        # index, label, ToA, pixel, ToT in; cluster record out
    "compact": (0, 64 + 64),     # cluster record in, feature row out
}


# Source files each kernel is built from (its counter record is void once any changes).
_COMMON = ["hc_device.h", "hc_internal.h", "hc_radix.h"]
KERNEL_SOURCES = {
    "tile_sort": ["hc_sort.hip"] + _COMMON, "tile_rank": ["hc_sort.hip"] + _COMMON,
    "link": ["hc_link.hip"] + _COMMON,
    "flatten": ["hc_link.hip"] + _COMMON, "features": ["hc_feat.hip"] + _COMMON,
    "compact": ["hc_feat.hip"] + _COMMON,
}
# Device function of each timed launch, as rocprofv3 names it.
KERNEL_FUNCS = {
    "tile_sort": "hc::k_tile_sort<", "tile_rank": "hc::k_tile_rank<",
    "link": "hc::k_link<", "flatten": "hc::k_flatten(", "features": "hc::k_features(",
    "compact": "hc::k_compact(",
}
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_mixed10m.json")


def kernel_sources_digest(kernel=None):
    """Digest of a kernel's source files (all of csrc when kernel is None)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2412_11809_amd", "csrc")
    files = KERNEL_SOURCES.get(kernel) if kernel else None
    for f in sorted(files or os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the kernel's current sources; else None."""
    try:
        data = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    rec = data.get("kernels", {}).get(kernel)
    if not rec or rec.get("sources") != kernel_sources_digest(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def _counter_values(path):
    """Per-dispatch counter values per (kernel name, counter), from the
    counter_collection.csv files rocprofv3 writes under `path`."""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        for row in csv.DictReader(open(f)):
            low = {k.lower(): v for k, v in row.items()}
            key = (low["kernel_name"], low["counter_name"])
            acc.setdefault(key, []).append(float(low["counter_value"]))
    return acc


def traffic_from(fetch_dir, write_dir, command):
    """Writes the counter summary: FETCH_SIZE / WRITE_SIZE (KiB per dispatch)
    per timed kernel, each scaled by what the counter reads for a plain 1 GiB
    device copy in the same run (bench.py --copy-calibration)."""
    fetch, write = _counter_values(fetch_dir), _counter_values(write_dir)

    def copy_reading(vals, counter):
        # the largest copy-kernel dispatch is the 1 GiB calibration copy
        got = [max(v) for (k, c), v in vals.items() if c == counter and "copyBuffer" in k]
        return max(got) if got else None

    f_copy, w_copy = copy_reading(fetch, "FETCH_SIZE"), copy_reading(write, "WRITE_SIZE")
    if not f_copy or not w_copy:
        raise SystemExit("no copy-kernel counter readings; run the profiled bench with --copy-calibration")
    f_scale, w_scale = (1 << 30) / (f_copy * 1024), (1 << 30) / (w_copy * 1024)
    out = {"command": command, "calibration": {"copy_bytes": 1 << 30, "fetch_kib": f_copy, "write_kib": w_copy,
                                               "fetch_scale": round(f_scale, 3), "write_scale": round(w_scale, 3)},
           "kernels": {}}
    for name, func in KERNEL_FUNCS.items():
        fk = [sum(v) / len(v) for (k, c), v in fetch.items() if c == "FETCH_SIZE" and func in k]
        wk = [sum(v) / len(v) for (k, c), v in write.items() if c == "WRITE_SIZE" and func in k]
        if not fk or not wk:
            continue
        fb, wb = fk[0] * 1024 * f_scale, wk[0] * 1024 * w_scale
        out["kernels"][name] = {"sources": kernel_sources_digest(name), "fetch_kib": round(fk[0], 1),
                                "write_kib": round(wk[0], 1), "hbm_bytes_per_launch": int(fb + wb)}
    json.dump(out, open(TRAFFIC_JSON, "w"), indent=1)
    print(json.dumps(out, indent=1))


def host_cpu():
    """CPU model and the cores this process may use (the box's share)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, usable, os.cpu_count()


def cpu_baseline(hits, p, sample_hits=4_000_000, runs=5):
    """The oracle (sequential, one core) on the first `sample_hits` hits of the
    workload (the paper's CPU benchmark also clusters 4M hits), median of
    `runs` runs; clustering only, generation excluded."""
    import oracle
    oracle.load()
    sample = hits[:sample_hits]
    n = sample.size
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.cluster(sample, p["width"], p["height"], p["dt"])
        ts.append(time.perf_counter() - t0)
    ts.sort()
    med = ts[len(ts) // 2]
    model, usable, total = host_cpu()
    return {"value": round(n / med / 1e6, 3), "unit": "Mhit/s", "cores": 1, "kind": "oracle",
            "sample": "the first %d hits of the 10M mixed workload, median of %d sequential runs "
                      "(%.2f s each; min %.2f, max %.2f)" % (n, runs, med, ts[0], ts[-1]),
            "cpu_model": model, "host_cores_usable": usable, "host_cores_total": total}


def cpu_lanes_baseline(hits, p, sample_hits=4_000_000, runs=3):
    """The paper's CPU method (temporal splitting over lanes, border merge
    cascade; cpu_lanes/) on the same sample as the oracle baseline, with one
    lane per usable host core: median of `runs` runs."""
    import cpu_lanes
    cpu_lanes.load()
    sample = hits[:sample_hits]
    model, usable, total = host_cpu()
    lanes = max(1, usable)
    window = 64 * p["dt"] * 512  # windows of ~5 ms at 10 Mhit/s
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        cpu_lanes.cluster(sample, p["width"], p["height"], p["dt"], lanes, window)
        ts.append(time.perf_counter() - t0)
    ts.sort()
    med = ts[len(ts) // 2]
    return {"value": round(sample.size / med / 1e6, 2), "unit": "Mhit/s", "cores": lanes, "kind": "cpu_lanes",
            "sample": "the first %d hits of the 10M mixed workload, median of %d runs (%.3f s)" % (
                sample.size, runs, med),
            "note": "the paper's multi-lane CPU clustering (temporal splitting, per-window sweep, merge cascade); "
                    "labels equal to the oracle's (tests/test_cpu_lanes.py)"}


# The paper's own figure for this path, with the hardware and clock it states.
PAPER_FIGURE = {
    "value": 300.0, "unit": "Mhit/s",
    "hardware": "NVIDIA RTX 4070 Ti Super 16 GB (PCIe 4.0 x16, 8848 cores) and RTX 3060 Laptop 6 GB "
                "(PCIe 4.0 x4, 3840 cores); the paper does not say which one reached the figure",
    "clock": "from a populated host buffer until the labels are back on the host (H2D and D2H included), "
             "warm-up excluded, timed from the second buffer",
    "workload": "the paper's measured datasets (not available here), so not the same workload as any line here",
    "source": "abstract and Section 5 (benchmarking results)"}


def bench_small(hc, torch, dev, calls=200):
    """The 100k-hit blob stream (a few clusters' worth of work per tile): one
    call costs about as much as its launches, so report call latency."""
    import hitgen
    hits, p = hitgen.blobs_100k()
    n = hits.size
    d = hc.hits_to_device(hits, dev)
    ws = torch.empty(hc.hc_workspace_size(n, p["width"], p["height"], p["disorder"]), dtype=torch.uint8, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    feats = torch.empty((n, 64), dtype=torch.uint8, device=dev)
    k = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def call():
        hc.hc_cluster(d, n, p["dt"], labels, feats, k, p["width"], p["height"], p["disorder"], ws, stream)

    for _ in range(10):
        call()
    torch.cuda.synchronize(dev)
    lat = []
    for _ in range(calls):
        t0 = time.perf_counter()
        call()
        torch.cuda.synchronize(dev)
        lat.append((time.perf_counter() - t0) * 1e3)
    t0 = time.perf_counter()
    for _ in range(calls):
        call()
    torch.cuda.synchronize(dev)
    back_to_back_ms = (time.perf_counter() - t0) * 1e3 / calls
    lat.sort()
    n_clusters = int(k.item())
    # the same call as a one-chunk batch captured in a HIP graph: one launch per call
    import numpy as np
    k1 = torch.empty(1, dtype=torch.int32, device=dev)
    graph = hc.hc_batch_graph_create(d, np.array([0, n], np.int64), np.array([p["dt"]], np.uint64), labels, feats,
                                     k1, None, p["width"], p["height"], p["disorder"])
    for _ in range(10):
        graph.launch(stream)
    torch.cuda.synchronize(dev)
    glat = []
    for _ in range(calls):
        t0 = time.perf_counter()
        graph.launch(stream)
        torch.cuda.synchronize(dev)
        glat.append((time.perf_counter() - t0) * 1e3)
    t0 = time.perf_counter()
    for _ in range(calls):
        graph.launch(stream)
    torch.cuda.synchronize(dev)
    graph_b2b_ms = (time.perf_counter() - t0) * 1e3 / calls
    assert int(k1.item()) == n_clusters, "graph replay cluster count differs"
    graph.close()
    glat.sort()
    return {"workload": "plain hc_cluster: 256x256 sensor, %d hits of random-walk blobs over 10 ms, "
                        "dt = 200 ns" % n,
            "n_hits": n, "n_clusters": n_clusters, "calls": calls,
            "latency_ms": {"p50": round(lat[len(lat) // 2], 4), "p99": round(lat[int(len(lat) * 0.99)], 4)},
            "back_to_back_ms_per_call": round(back_to_back_ms, 4),
            "graph_latency_ms": {"p50": round(glat[len(glat) // 2], 4), "p99": round(glat[int(len(glat) * 0.99)], 4)},
            "graph_back_to_back_ms_per_call": round(graph_b2b_ms, 4),
            "note": "latency = one call from the host until its results are on the device, synchronised; "
                    "graph = the same call captured once as a one-chunk batch and replayed"}


def bench_batch(hc, torch, dev, reps):
    """64 chunks of log-uniform size (~27M hits, 4 detectors, dt per chunk in
    {100, 200, 500} ns): the plain path chunk after chunk vs one batched launch
    sequence (default plan, autotuned plan, and its HIP-graph replay)."""
    import numpy as np
    import hitgen
    chunks, dts, _ = hitgen.batch_64_chunks()
    sizes = np.array([c.size for c in chunks], dtype=np.int64)
    offsets = np.zeros(len(chunks) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    n = int(offsets[-1])
    dts = np.asarray(dts, dtype=np.uint64)
    d_hits = hc.hits_to_device(np.concatenate(chunks), dev)
    del chunks
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    feats = torch.empty((n, 64), dtype=torch.uint8, device=dev)
    k = torch.empty(len(sizes), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    hint = 512
    ws = torch.empty(hc.hc_workspace_size(int(sizes.max()), 256, 256, hint), dtype=torch.uint8, device=dev)
    views = [(d_hits[16 * offsets[c]:16 * offsets[c + 1]], labels[offsets[c]:offsets[c + 1]],
              feats[offsets[c]:offsets[c + 1]], k[c:c + 1]) for c in range(len(sizes))]

    def sequential():
        for c, (h, l, f, kk) in enumerate(views):
            hc.hc_cluster(h, int(sizes[c]), int(dts[c]), l, f, kk, 256, 256, hint, ws, stream)

    def timed(fn):
        fn()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize(dev)
        return (time.perf_counter() - t0) / reps

    t_seq = timed(sequential)
    k_seq = k.cpu().numpy().copy()
    t_def = timed(lambda: hc.hc_cluster_batch(d_hits, offsets, dts, labels, feats, k, None, 256, 256, hint,
                                              None, stream))
    assert np.array_equal(k.cpu().numpy(), k_seq), "batched and sequential cluster counts differ"
    t0 = time.perf_counter()
    plan = hc.hc_batch_autotune(d_hits, offsets, dts, labels, feats, k, 256, 256, hint, stream)
    torch.cuda.synchronize(dev)
    t_tune = time.perf_counter() - t0
    t_plan = timed(lambda: hc.hc_cluster_batch(d_hits, offsets, dts, labels, feats, k, plan, 256, 256, hint,
                                               None, stream))
    graph = hc.hc_batch_graph_create(d_hits, offsets, dts, labels, feats, k, plan, 256, 256, hint)
    t_graph = timed(lambda: graph.launch(stream))
    assert np.array_equal(k.cpu().numpy(), k_seq), "graph replay cluster counts differ"
    desc = plan.describe()
    graph.close()
    plan.close()
    mh = lambda t: round(n / t / 1e6, 1)
    return {"workload": "64 chunks, log-uniform sizes in [1k, 2M] (%d hits), 4 detectors of 256x256, "
                        "dt per chunk in {100, 200, 500} ns, local shuffle <= 512" % n,
            "n_hits": n, "n_clusters": int(k_seq.sum()), "reps": reps,
            "plain_sequential_mhits": mh(t_seq), "batched_mhits": mh(t_def),
            "batched_autotuned_mhits": mh(t_plan), "batched_graph_mhits": mh(t_graph),
            "speedup_vs_plain": round(t_seq / min(t_plan, t_graph, t_def), 2),
            "plan": desc, "autotune_s": round(t_tune, 2),
            "ms": {"plain_sequential": round(t_seq * 1e3, 3), "batched": round(t_def * 1e3, 3),
                   "autotuned": round(t_plan * 1e3, 3), "graph": round(t_graph * 1e3, 3)}}


def bench_stream(hc, torch, dev, n_total=200_000_000, chunk=1_000_000):
    """The Timepix4-shaped stream (448x512, 300 Mhit/s, 195.3125 ps ticks,
    blobs of min(60, Geom(mean 9)) hits, displacement <= 16384, dt = 200 ns)
    pushed through one hc_stream as consecutive 1M-hit chunks from HBM, open
    clusters stitched on the device.  The first push is a warm-up (the paper
    times from its second buffer on); the rate covers every later push and
    the flush.  Closed features are drained to pinned host memory between
    pushes (inside the timed span, overlapping the pushes in flight)."""
    import numpy as np
    import hitgen
    p = hitgen.TPX4_PARAMS
    workers = min(16, host_cpu()[1] or 1)
    d_hits = torch.empty(16 * n_total, dtype=torch.uint8, device=dev)
    at, run_max, tdis = 0, 0, 0
    t_gen = time.perf_counter()
    for piece in hitgen.timepix4_stream(n_total, workers=workers):
        m = piece.size
        d_hits[16 * at:16 * (at + m)].copy_(torch.from_numpy(piece.view(np.uint8).reshape(-1)))
        t = piece["toa"].astype(np.int64)
        before = np.maximum(np.concatenate([[run_max], np.maximum.accumulate(t)[:-1]]), run_max)
        tdis = max(tdis, int((before - t).max()))
        run_max = max(run_max, int(t.max()))
        at += m
    t_gen = time.perf_counter() - t_gen
    assert at == n_total
    print("stream workload generated (%.1f s)" % t_gen, file=sys.stderr, flush=True)
    labels = torch.full((n_total,), -1, dtype=torch.int32, device=dev)
    st = hc.HcStream(p["dt"], tdis + 1, p["width"], p["height"], p["disorder"])
    st.reserve(chunk)
    open_hw, n_closed = 0, 0
    t_push, lat_ms = {}, []

    def take(tags, k):
        nonlocal n_closed
        now = time.perf_counter()
        for tg in tags:
            lat_ms.append((now - t_push.pop(tg)) * 1e3)
        n_closed += k

    n_chunks = (n_total + chunk - 1) // chunk
    t_start = None
    for c in range(n_chunks):
        a, b = c * chunk, min(n_total, (c + 1) * chunk)
        t_push[c] = time.perf_counter()
        st.hc_stream_push(d_hits[16 * a:16 * b], b - a, labels[a:b], c)
        if c == 0:  # warm-up push, excluded from the rate
            st.wait()
            t_start = time.perf_counter()
        open_hw = max(open_hw, st.open_hits())
        take(*st.drain())
    st.flush()
    torch.cuda.synchronize(dev)
    t_end = time.perf_counter()
    take(*st.drain())
    rejected = dict(st.rejected)
    st.close()
    assert not rejected, "chunks rejected: %s" % rejected
    assert not t_push, "not every chunk completed"
    assert int((labels < 0).sum().item()) == 0, "labels left unwritten"
    timed_hits = n_total - min(chunk, n_total)
    lat = np.array(lat_ms[1:]) if len(lat_ms) > 1 else np.array(lat_ms)
    return {"workload": "Timepix4-shaped 448x512 sensor, %d hits at 300 Mhit/s (195.3125 ps ticks), blobs of "
                        "min(60, Geom(mean 9)) hits, local shuffle <= 16384, dt = 200 ns = 1024 ticks, pushed as "
                        "%d-hit chunks through one hc_stream (exact stitching on the device)" % (n_total, chunk),
            "n_hits": n_total, "chunks": n_chunks, "n_clusters": n_closed, "max_disorder_ticks": tdis + 1,
            "mhits": round(timed_hits / (t_end - t_start) / 1e6, 1),
            "ms_total": round((t_end - t_start) * 1e3, 2),
            "chunk_final_latency_ms": {"p50": round(float(np.quantile(lat, 0.5)), 3),
                                       "p99": round(float(np.quantile(lat, 0.99)), 3)},
            "open_hits_high_water": open_hw, "generation_s": round(t_gen, 1),
            "note": "device-resident: hits in HBM before the first push, labels written to HBM, closed features "
                    "drained to the host between pushes; rate = hits of pushes 2..%d over the wall time from "
                    "the second push to the end of the flush; latency = push call to the chunk's labels all "
                    "final (seen by the next poll)" % n_chunks}


def bench_variants(hc, torch, dev, hits, p, reps=3):
    """On the 10M mixed stream (resident in HBM): the Section 2 (iii)(b)
    clustering (HC_FLAG_GLOBAL_TIME), and the per-cluster products of a
    default clustering (boxes, a size filter, the kept hits grouped cluster by
    cluster).  Mean of `reps` timed calls after one warm-up."""
    import numpy as np
    n = hits.size
    W, H, dt, D = p["width"], p["height"], p["dt"], p["disorder"]
    d = hc.hits_to_device(hits, dev)
    stream = torch.cuda.current_stream(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    feats = torch.empty((n, 64), dtype=torch.uint8, device=dev)
    k = torch.empty(1, dtype=torch.int32, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize(dev)
        return (time.perf_counter() - t0) / reps

    ws_g = torch.empty(hc.hc_workspace_size(n, W, H, D, hc.HC_FLAG_GLOBAL_TIME), dtype=torch.uint8, device=dev)
    t_g = timed(lambda: hc.hc_cluster(d, n, dt, labels, feats, k, W, H, D, ws_g, stream, hc.HC_FLAG_GLOBAL_TIME))
    k_g = int(k.item())
    del ws_g
    ws = torch.empty(hc.hc_workspace_size(n, W, H, D), dtype=torch.uint8, device=dev)
    t_a = timed(lambda: hc.hc_cluster(d, n, dt, labels, feats, k, W, H, D, ws, stream))
    k_a = int(k.item())
    boxes = torch.empty((n, 8), dtype=torch.uint8, device=dev)
    keep = torch.empty(n, dtype=torch.int32, device=dev)
    nkeep = torch.empty(1, dtype=torch.int32, device=dev)
    grouped = torch.empty((n, 16), dtype=torch.uint8, device=dev)
    gidx = torch.empty(n, dtype=torch.int32, device=dev)
    start = torch.empty(n + 1, dtype=torch.int64, device=dev)
    pws = torch.empty(hc.hc_products_workspace_size(n), dtype=torch.uint8, device=dev)
    flt = {"min_size": 3}
    t_p = timed(lambda: hc.hc_cluster_products(d, n, labels, feats, k, keep, nkeep, boxes=boxes, grouped=grouped,
                                               grouped_idx=gidx, row_start=start, filter=flt, workspace=pws,
                                               stream=stream))
    t_b = timed(lambda: hc.hc_cluster_products(d, n, labels, feats, k, keep, nkeep, boxes=boxes, workspace=pws,
                                               stream=stream))
    return {"workload": "the 10M mixed stream of the plain line, resident in HBM",
            "global_time_iii_b": {"mhits": round(n / t_g / 1e6, 1), "ms": round(t_g * 1e3, 3), "n_clusters": k_g,
                                  "n_clusters_iii_a": k_a,
                                  "note": "Section 2 (iii)(b) clusters; the host waits for every refinement round"},
            "products": {"ms_boxes_filter_grouping": round(t_p * 1e3, 3), "ms_boxes_filter": round(t_b * 1e3, 3),
                         "kept_clusters": int(nkeep.item()), "filter": "size >= 3",
                         "note": "after a plain clustering of the same hits; grouping = the kept clusters' hits "
                                 "in cluster-major order (stable radix sort)"}}


def bench_showers(hc, torch, dev, n=10_000_000, reps=5):
    """Plain calls on streams with dense showers (hitgen.shower_stream: 30 %
    of the hits in showers of U{lo..hi} hits within 100 ns), where many link
    tiles have more than 1024 hits within dt before them: the moderate case
    is handled by the wide second level tile by tile, the deep one partly by
    the all-hits fallback.  Mean of `reps` timed calls after one warm-up, and
    the link kernels' share from HIP events in a separate call."""
    import hitgen
    out = {"workload": "256x256 sensor, %d hits at ~10 Mhit/s (the mixed stream plus dense showers: 30 %% of "
                       "the hits in showers within 100 ns), local shuffle <= 4096, dt = 128 ticks" % n}
    for name, sizes in (("showers_1500_6000", (1500, 6000)), ("showers_9000_14000", (9000, 14000))):
        hits = hitgen.shower_stream(n, hitgen.BASE_SEED + 60 + sizes[0], shower_hits=sizes)
        d = hc.hits_to_device(hits, dev)
        stream = torch.cuda.current_stream(dev)
        ws = torch.empty(hc.hc_workspace_size(n, 256, 256, 4096), dtype=torch.uint8, device=dev)
        labels = torch.empty(n, dtype=torch.int32, device=dev)
        feats = torch.empty((n, 64), dtype=torch.uint8, device=dev)
        k = torch.empty(1, dtype=torch.int32, device=dev)

        def call():
            hc.hc_cluster(d, n, 128, labels, feats, k, 256, 256, 4096, ws, stream)

        call()
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize(dev)
        tm = (time.perf_counter() - t0) / reps
        hc.hc_timing_reset()
        hc.hc_timing_enable(True)
        call()
        torch.cuda.synchronize(dev)
        hc.hc_timing_enable(False)
        kt = hc.hc_timing_read()
        out[name] = {"mhits": round(n / tm / 1e6, 1), "ms": round(tm * 1e3, 3), "n_clusters": int(k.item()),
                     "link_ms": {kn: round(kt[kn][1], 4) for kn in ("link", "link_wide", "link_fallback")
                                 if kn in kt}}
        del d, ws, labels, feats
        torch.cuda.empty_cache()
    return out


def bench_ingest(hc, torch, dev, hits, p, piece=65536, reps=3):
    """The host ingest front end on the paper's clock: the hits start in a
    host array (the populated host buffer) and are fed in arrival order in
    pieces of `piece` hits; buffers of b = 256k hits are filled by the
    paper's buffer filling (b_t = 16k: at most 13.9k hits of this stream
    arrive within t + t_closing), copied to the device (pinned, on their own
    stream), clustered with exact stitching, and every label ends on the host
    at its arrival index.  One untimed warm-up run, then the mean of `reps`
    runs.  (Buffers of 2M or 8M hits make the host's filling about twice as
    slow on this machine.)"""
    import numpy as np
    import hitgen
    n = hits.size
    t = hitgen.realised_disorder_ticks(hits) + 1
    b, bt = 256 << 10, 16 << 10
    labels = torch.empty(n, dtype=torch.int32, pin_memory=True)
    src = np.ascontiguousarray(hits)
    times, st = [], None
    for r in range(reps + 1):
        ing = hc.HcIngest(labels, p["dt"], t, 64 * p["dt"], b, bt, p["width"], p["height"], p["disorder"])
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        for a in range(0, n, piece):
            ing.feed(src[a:a + piece])
        ing.finish()
        t1 = time.perf_counter()
        st = ing.stats()
        ing.close()
        if r:
            times.append(t1 - t0)
    ok = int((labels.numpy() >= 0).all())
    tm = sum(times) / len(times)
    return {"workload": "the 10M mixed stream of the plain line, fed from host memory in arrival order, pieces of "
                        "%d hits; buffers b = %d, b_t = %d, t_closing = 64 dt" % (piece, b, bt),
            "mhits": round(n / tm / 1e6, 1), "ms": round(tm * 1e3, 2), "reps": reps,
            "buffers_sent": st["buffers_sent"], "diverted_hits": st["diverted"], "labels_complete": bool(ok),
            "note": "end-to-end: buffer filling on the host, host-to-device copy, clustering, labels back at their "
                    "arrival indices; warm-up run excluded"}


def _served_pools(n_streams, pool, seed):
    """One pool of random-walk blobs at 37.5 Mhit/s per stream; stream s sees it
    under the s-th symmetry of the square sensor (so the streams differ)."""
    import numpy as np
    import hitgen
    span = int(round(pool / 37.5e6 * 1e9 / hitgen.TPX3_TICK_NS))
    base = hitgen.blob_stream(pool, seed, 256, 256, span_ticks=span, jitter=hitgen.ns_to_ticks(100, hitgen.TPX3_TICK_NS),
                              disorder=512)
    pools = []
    for s in range(n_streams):
        h = base.copy()
        x, y = base["x"].astype(np.int32), base["y"].astype(np.int32)
        if s & 1:
            x = 255 - x
        if s & 2:
            y = 255 - y
        if s & 4:
            x, y = y, x
        h["x"], h["y"] = x, y
        pools.append(h)
    return pools, int(base["toa"].max()) + 1, hitgen.realised_disorder_ticks(base) + 1


def _chunk_plan(rng, n, lo=4000, hi=1_000_000):
    import numpy as np
    sizes = []
    left = n
    while left > 0:
        m = min(left, int(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        sizes.append(m)
        left -= m
    return sizes


def bench_served(hc, torch, dev, seconds, n_streams=8, pool=4_000_000, rate_mhits=300.0, check_pass=None,
                 rate_only=False):
    """8 detector streams (256x256, 37.5 Mhit/s each), chunks of log-uniform
    size in [4k, 1M] hits arriving as independent Poisson processes at an
    aggregate 300 Mhit/s, HBM budget 16 GiB, dt = 200 ns.  Each stream replays
    its pool with a ToA offset per pass (two pinned copies, re-offset in place
    once a pass has completed).  Also: the saturated rate (every chunk of one
    pass submitted at once) against the same chunks pushed one by one through
    one stream at a time.

    check_pass(stream, pass_index, n_hits, labels) -- optional, for tests: is
    called with the final labels (a host int32 array) of the first n_hits hits
    of every pass of the rate-limited run once they are all final.
    rate_only -- skip the saturated and one-stream-at-a-time measurements."""
    import heapq
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import hitgen
    seed = hitgen.BASE_SEED + 5
    pools, span, tdis = _served_pools(n_streams, pool, seed)
    period = span + tdis + 4096  # ToA offset between passes
    dt = 128
    rng = np.random.default_rng([seed, 9])

    def pinned_hits(a):
        t = torch.empty(a.nbytes, dtype=torch.uint8, pin_memory=True)
        v = t.numpy().view(hitgen.HIT_DTYPE)
        v[:] = a
        return t, v

    copies = [[pinned_hits(p) for _ in range(2)] for p in pools]
    labels = [[torch.empty(pool, dtype=torch.int32, pin_memory=True) for _ in range(2)] for _ in pools]

    plans = [_chunk_plan(rng, pool) for _ in range(n_streams)]  # drawn either way: same later chunks
    # chunks per second per stream for the offered hit rate: a pass of the
    # pool ends with a shortened chunk, so the mean chunk is that of the plans
    # (estimated over 2000 of them, on a generator of its own)
    sim = np.random.default_rng([seed, 11])
    mean_chunk = pool * 2000 / sum(len(_chunk_plan(sim, pool)) for _ in range(2000))
    lam = rate_mhits * 1e6 / n_streams / mean_chunk
    sat = None
    if not rate_only:
        sat_mhits, seq_mhits, sat = _served_saturated(hc, torch, dev, n_streams, pool, dt, tdis, copies, labels,
                                                      plans, pools, period)

    # -- rate-limited: Poisson arrivals at the aggregate rate for `seconds`

    srv = hc.HcServer(n_streams, dt, tdis, hbm_budget=16 << 30, disorder_hint=512)
    import threading
    read_stop, closed_read = threading.Event(), [0]
    reader = threading.Thread(target=_read_closed, args=(srv, n_streams, np.zeros(1 << 16, dtype=hc.FEATURE_DTYPE),
                                                         read_stop, closed_read))
    reader.start()
    ex = ThreadPoolExecutor(max_workers=4)
    ready = [[None, None] for _ in range(n_streams)]   # future of the in-place re-offset
    passes = [[0, 1] for _ in range(n_streams)]        # pass held by each copy
    outstanding = [[0, 0] for _ in range(n_streams)]
    submitted = [[0, 0] for _ in range(n_streams)]      # hits of the held pass submitted so far
    state = [{"pass": 0, "plan": _chunk_plan(rng, pool), "c": 0, "at": 0} for _ in range(n_streams)]
    # the second copy starts one period later
    for s in range(n_streams):
        copies[s][1][1]["toa"] += np.uint64(period)
    start = hc.hc_server_now_ns() + 20_000_000
    end = start + int(seconds * 1e9)
    events = [(start + int(rng.exponential(1e9 / lam)), s) for s in range(n_streams)]
    heapq.heapify(events)
    key_of = {}
    n_sub = 0
    comps = []

    def collect():
        for c in srv.poll(1 << 14):
            s, cp = key_of.pop((int(c["stream_id"]), int(c["tag"])))
            outstanding[s][cp] -= 1
            comps.append(c)

    while events and events[0][0] < end:
        t_arr, s = heapq.heappop(events)
        while hc.hc_server_now_ns() < t_arr:
            collect()
            time.sleep(0.0002)
        stt = state[s]
        cp = stt["pass"] % 2
        if passes[s][cp] != stt["pass"]:
            # wait until this copy's previous pass has completed, then re-offset it
            while outstanding[s][cp] > 0:
                collect()
                time.sleep(0.0002)
            if check_pass is not None and submitted[s][cp]:
                check_pass(s, passes[s][cp], submitted[s][cp], labels[s][cp].numpy())
            submitted[s][cp] = 0
            if ready[s][cp] is None:
                v = copies[s][cp][1]
                ready[s][cp] = ex.submit(lambda v=v: v["toa"].__iadd__(np.uint64(2 * period)))
            ready[s][cp].result()
            ready[s][cp] = None
            passes[s][cp] = stt["pass"]
        m = stt["plan"][stt["c"]]
        at = stt["at"]
        tag = n_sub
        key_of[(s, tag)] = (s, cp)
        outstanding[s][cp] += 1
        submitted[s][cp] += m
        srv.submit(s, copies[s][cp][0][16 * at:16 * (at + m)], labels[s][cp][at:at + m], tag, t_arr)
        n_sub += 1
        stt["c"] += 1
        stt["at"] += m
        if stt["c"] == len(stt["plan"]):
            stt.update({"pass": stt["pass"] + 1, "plan": _chunk_plan(rng, pool), "c": 0, "at": 0})
        heapq.heappush(events, (t_arr + int(rng.exponential(1e9 / lam)), s))
    t_last_arrival = hc.hc_server_now_ns()
    srv.wait_idle(600000)
    for s in range(n_streams):
        srv.flush(s)
    srv.wait_idle(600000)
    collect()
    read_stop.set()
    reader.join()
    if check_pass is not None:
        for s in range(n_streams):
            for cp in range(2):
                if submitted[s][cp]:
                    check_pass(s, passes[s][cp], submitted[s][cp], labels[s][cp].numpy())
    stats = srv.stats()
    srv.close()
    ex.shutdown()
    comps = np.array(comps, dtype=hc.COMPLETION_DTYPE) if comps else np.empty(0, dtype=hc.COMPLETION_DTYPE)
    ok = comps[comps["status"] == 0]
    hits_done = int(ok["n_hits"].sum())
    t_span = (int(ok["t_final_ns"].max()) - start) / 1e9 if ok.size else float("nan")
    proc = (ok["t_processed_ns"] - ok["t_arrive_ns"]) / 1e6
    fin = (ok["t_final_ns"] - ok["t_arrive_ns"]) / 1e6
    q = lambda a, f: round(float(np.quantile(a, f)), 3) if a.size else None
    out = {"workload": "%d streams of 256x256 at %.1f Mhit/s each, Poisson chunk arrivals (aggregate %.0f Mhit/s), "
                       "chunks log-uniform in [4k, 1M] hits, dt = 200 ns, HBM budget 16 GiB, pools of %d hits "
                       "replayed with a ToA offset per pass" % (n_streams, rate_mhits / n_streams, rate_mhits, pool),
           "seconds": seconds, "chunks": int(comps.size), "rejected": int((comps["status"] != 0).sum()),
           "hits_served": hits_done, "closed_clusters_read": int(closed_read[0]),
           "offered_mhits": rate_mhits, "offered_chunks_per_s": round(lam * n_streams, 1),
           "achieved_mhits": round(hits_done / t_span / 1e6, 1),
           "processing_latency_ms": {"p50": q(proc, 0.5), "p99": q(proc, 0.99)},
           "final_latency_ms": {"p50": q(fin, 0.5), "p99": q(fin, 0.99)},
           "hbm_peak_bytes": int(stats["hbm_peak"]), "peak_slots_in_use": int(stats["peak_slots_in_use"]),
           "note": "end-to-end from pinned host memory (H2D hits, D2H labels and closed features); a client "
                   "thread reads the closed clusters' features as they come"}
    if sat is not None:
        out.update({"saturated_mhits": round(sat_mhits, 1), "one_stream_at_a_time_mhits": round(seq_mhits, 1),
                    "saturated_speedup": round(sat_mhits / seq_mhits, 2),
                    "saturated_hbm_peak_bytes": int(sat["hbm_peak"]),
                    "saturated_pass_mhits": sat["pass_mhits"], "saturated_pushes": int(sat["pushes"]),
                    "saturated_chunks": sum(len(p) for p in plans),
                    "saturated_worker_ms": {k: round(sat[k] / 1e6, 2) for k in ("ns_admit_wait", "ns_push",
                                                                               "ns_drain", "ns_final")}})
    return out


def _read_closed(srv, n_streams, buf, stop, got):
    """A server's client: reads every stream's closed-cluster features into
    one reused buffer until `stop` is set, then once more; got[0] counts them."""
    while True:
        last = stop.is_set()
        moved = 0
        for s in range(n_streams):
            while True:
                k = srv.closed_into(s, buf)
                moved += k
                if k < buf.size:
                    break
        got[0] += moved
        if last:
            return
        if moved == 0:
            time.sleep(0.0002)


def _served_saturated(hc, torch, dev, n_streams, pool, dt, tdis, copies, labels, plans, pools, period, passes=5):
    """One pass of every stream submitted to the server at once (saturated
    rate), on one server that stays up across the passes as a service would,
    so its device buffers are allocated in the untimed warm-up pass; the
    median of `passes` timed passes, pass k replaying the pools k periods
    later (each stream is flushed at the end of a pass).  A consumer thread
    reads the closed clusters' features while the pass runs, as the service's
    client would (the server reuses the blocks it has read out), and the
    count it read is checked against the chunks' closed counts.  Then the same chunks
    pushed through one hc_stream at a time."""
    import threading
    import numpy as np
    rates, sats = [], []
    buf = np.zeros(1 << 16, dtype=hc.FEATURE_DTYPE)  # the consumer's reused buffer
    consume = lambda srv, stop, got: _read_closed(srv, n_streams, buf, stop, got)

    keys = ("pushes", "ns_admit_wait", "ns_push", "ns_drain", "ns_final")
    srv = hc.HcServer(n_streams, dt, tdis, hbm_budget=16 << 30, disorder_hint=512)
    prev = {k: 0 for k in keys}
    done = 0
    for rep in range(passes + 1):
        cp = rep % 2  # last read two passes ago; every pass has completed before the next
        for s in range(n_streams):
            copies[s][cp][1]["toa"] = pools[s]["toa"] + np.uint64(rep * period)
        stop, got = threading.Event(), [0]
        reader = threading.Thread(target=consume, args=(srv, stop, got))
        reader.start()
        t0 = hc.hc_server_now_ns()
        for s in range(n_streams):
            at = 0
            for c, m in enumerate(plans[s]):
                srv.submit(s, copies[s][cp][0][16 * at:16 * (at + m)], labels[s][cp][at:at + m], c, t0)
                at += m
        for s in range(n_streams):
            srv.flush(s)
        srv.wait_idle(600000)
        t1 = hc.hc_server_now_ns()
        stop.set()
        reader.join()
        comp = srv.poll(1 << 16)
        st = srv.stats()
        assert (comp["status"] == 0).all() and comp.size == sum(len(p) for p in plans)
        # at least the chunks' closed clusters (those the end-of-pass flushes
        # close belong to no chunk)
        assert got[0] >= int(comp["n_closed"].sum()) > 0, (got[0], int(comp["n_closed"].sum()))
        done += comp.size
        if rep:
            rates.append(n_streams * pool / ((t1 - t0) / 1e9) / 1e6)
            sats.append(dict(st, **{k: st[k] - prev[k] for k in keys}))
        prev = {k: st[k] for k in keys}
    srv.close()
    for s in range(n_streams):  # both copies back at the pools' own ToAs
        for cp in range(2):
            copies[s][cp][1]["toa"] = pools[s]["toa"]
    order = sorted(range(passes), key=lambda i: rates[i])
    sat_mhits, sat = rates[order[passes // 2]], sats[order[passes // 2]]
    sat["pass_mhits"] = [round(r, 1) for r in rates]

    t0 = time.perf_counter()
    for s in range(n_streams):
        st = hc.HcStream(dt, tdis, 256, 256, 512)
        st.reserve(1_000_000)
        d_hits = torch.empty(16 * 1_000_000, dtype=torch.uint8, device=dev)
        d_lab = [torch.empty(1_000_000, dtype=torch.int32, device=dev) for _ in range(len(plans[s]))]
        at = 0
        for c, m in enumerate(plans[s]):
            d_hits[:16 * m].copy_(copies[s][0][0][16 * at:16 * (at + m)], non_blocking=True)
            st.hc_stream_push(d_hits, m, d_lab[c], c)
            st.poll()
            at += m
        st.flush()
        st.poll()
        torch.cuda.synchronize(dev)
        st.close()
    seq_mhits = n_streams * pool / (time.perf_counter() - t0) / 1e6
    return sat_mhits, seq_mhits, sat


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--hits", type=int, default=10_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch-form measurement")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--served-seconds", type=float, default=10.0)
    ap.add_argument("--no-stream", action="store_true", help="skip the Timepix4 stream measurement")
    ap.add_argument("--no-extras", action="store_true", help="skip the variant, products and ingest measurements")
    ap.add_argument("--stream-hits", type=int, default=200_000_000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--only", choices=["plain", "batch", "served", "stream"],
                    help="run one form only (profiling runs); the plain line is still printed")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_mixed10m.json from two rocprofv3 --pmc runs (CSV output) "
                         "of this bench with --copy-calibration, then exit")
    ap.add_argument("--traffic-command", default="", help="the profiling command, recorded in the summary")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(args.traffic_from[0], args.traffic_from[1], args.traffic_command)
        return
    if args.only == "plain":
        args.no_batch = args.no_served = args.no_stream = args.no_extras = True
    elif args.only in ("batch", "served", "stream"):
        args.steps, args.warmup = 1, 0
        args.no_batch, args.no_served = args.only != "batch", args.only != "served"
        args.no_stream = args.only != "stream"
        args.no_extras = True
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import hitgen
    import paper_2412_11809_amd as hc

    hc.load_library()
    hits, p = hitgen.mixed_10m(n=args.hits)
    n = hits.size
    W, H, dt, D = p["width"], p["height"], p["dt"], p["disorder"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # two copies of the input (320 MB together), used in turn, so the hit
    # records cannot stay resident in the 256 MB Infinity Cache between steps
    d_hits = [hc.hits_to_device(hits, dev)]
    d_hits.append(d_hits[0].clone())
    ws = torch.empty(hc.hc_workspace_size(n, W, H, D), dtype=torch.uint8, device=dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    feats = torch.empty((n, 64), dtype=torch.uint8, device=dev)
    k = torch.empty(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step(i):
        hc.hc_cluster(d_hits[i & 1], n, dt, labels, feats, k, W, H, D, ws, stream)

    # warm-up steps: every kernel bracketed by HIP events (after the first
    # step), which gives the per-kernel breakdown and the dominant kernel
    breakdown, n_break = {}, 0
    for i in range(args.warmup):
        if i == min(1, args.warmup - 1):
            torch.cuda.synchronize(dev)
            hc.hc_timing_reset()
            hc.hc_timing_enable(True)
            n_break = args.warmup - i
        step(i)
    torch.cuda.synchronize(dev)
    hc.hc_timing_enable(False)
    if n_break:
        breakdown = hc.hc_timing_read()
    print("warmup done", file=sys.stderr, flush=True)
    dom = max(breakdown, key=lambda name: breakdown[name][1]) if breakdown else "link"

    # timed steps: events on the dominant kernel's launches only, so the other
    # launches run exactly as they do without measurement
    hc.hc_timing_reset()
    hc.hc_timing_select(dom)
    hc.hc_timing_enable(True)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    hc.hc_timing_enable(False)
    hc.hc_timing_select(None)
    times = hc.hc_timing_read()
    n_clusters = int(k.item())
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e6

    launches, total_ms = times[dom]
    avg_ms = total_ms / launches
    # the path's algorithmic bytes (read every 16-byte hit once, write its
    # 4-byte label, write one 64-byte feature row per cluster) over the
    # dominant kernel's duration; the kernel's own contract bytes beside it
    path_bytes = 20 * n + 64 * n_clusters
    achieved = path_bytes / (avg_ms / 1e3) / 1e9
    per_hit, per_cluster = ALG_BYTES.get(dom, (0, 0))
    contract = per_hit * n + per_cluster * n_clusters
    traffic = measured_traffic(dom)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mhit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain hc_cluster: 256x256 Timepix3 sensor, %d hits (~10 Mhit/s over ~1 s: "
                               "70%% small blobs, 25%% tracks, 5%% heavy blobs), local shuffle <= 4096, "
                               "dt = 200 ns = 128 ticks" % n,
                   "n_hits": n, "n_clusters": n_clusters, "form": "plain"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel_avg_ms": round(avg_ms, 4), "alg_bytes_per_launch": path_bytes,
                     "kernel_contract_frac": round(contract / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "path_roofline": {"achieved": round(path_bytes / (ms_per_step / 1e3) / 1e9, 1), "unit": "GB/s",
                          "frac": round(path_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                          "bytes_per_step": path_bytes},
        "kernels_ms_per_step": {name: round(v[1] / n_break, 4) for name, v in sorted(breakdown.items())},
        "sources": kernel_sources_digest(),
        "paper": PAPER_FIGURE,
    }
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        out["copy_calibration_bytes"] = 1 << 30
    if args.only is None:
        out["small"] = bench_small(hc, torch, dev)
        print("small done", file=sys.stderr, flush=True)
    if not args.no_extras:
        out["variants"] = bench_variants(hc, torch, dev, hits, p)
        print("variants done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["ingest"] = bench_ingest(hc, torch, dev, hits, p)
        print("ingest done", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["showers"] = bench_showers(hc, torch, dev)
        print("showers done", file=sys.stderr, flush=True)
    if not args.no_batch:
        del d_hits, ws, labels, feats
        torch.cuda.empty_cache()
        out["batch"] = bench_batch(hc, torch, dev, reps=5)
        print("batch done", file=sys.stderr, flush=True)
    if not args.no_served:
        torch.cuda.empty_cache()
        out["served"] = bench_served(hc, torch, dev, args.served_seconds)
        print("served done", file=sys.stderr, flush=True)
    if not args.no_stream:
        torch.cuda.empty_cache()
        out["stream"] = bench_stream(hc, torch, dev, n_total=args.stream_hits)
        print("stream done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(hits, p)
        out["cpu_lanes"] = cpu_lanes_baseline(hits, p)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
