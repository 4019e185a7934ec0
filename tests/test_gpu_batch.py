"""GPU parity of the batch form: every chunk of a batch must get exactly the
labels, features and cluster count the oracle gives that chunk alone; the
autotuned plan and the captured graph must reproduce the eager result."""
import numpy as np
import pytest

import hitgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2412_11809_amd as hc
    assert torch.cuda.is_available()
    hc.load_library()
    return hc


def pack(chunks):
    offsets = np.zeros(len(chunks) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([c.size for c in chunks])
    hits = np.concatenate(chunks) if offsets[-1] else np.empty(0, dtype=hitgen.HIT_DTYPE)
    return hits, offsets


def fetch(hc, labels, feats, k, offsets):
    """Device outputs -> per-chunk (labels, features) lists and the counts."""
    k = k.cpu().numpy()
    lab = labels.cpu().numpy()
    fb = feats.cpu().numpy().reshape(-1).view(hc.FEATURE_DTYPE) if feats is not None else None
    out = []
    for c in range(len(offsets) - 1):
        a, b = offsets[c], offsets[c + 1]
        f = fb[a:a + max(int(k[c]), 0)].copy() if fb is not None else None
        out.append((lab[a:b].copy(), f))
    return out, k


def expect(chunks, dts, w=256, h=256):
    return [oracle.cluster(c, w, h, int(dt)) for c, dt in zip(chunks, dts)]


def compare(got, k, want, tag=""):
    for c, ((gl, gf), (wl, wf)) in enumerate(zip(got, want)):
        assert k[c] == wf.size, "%s chunk %d: %d clusters, oracle %d" % (tag, c, k[c], wf.size)
        bad = np.nonzero(gl != wl)[0]
        assert bad.size == 0, "%s chunk %d: %d labels differ, first %s: %s vs %s" % (
            tag, c, bad.size, bad[:5], gl[bad[:5]], wl[bad[:5]])
        if gf is not None:
            assert gf.tobytes() == wf.tobytes(), "%s chunk %d: features differ" % (tag, c)


def run(hc, chunks, dts, plan=None, hint=0, features=True):
    import torch
    hits, offsets = pack(chunks)
    print("batch case: chunks=%d n=%d hint=%d" % (len(chunks), offsets[-1], hint), flush=True)
    d = hc.hits_to_device(hits) if hits.size else torch.empty(16, dtype=torch.uint8, device="cuda")
    labels, feats, k = hc.cluster_batch(d, offsets, np.asarray(dts, dtype=np.uint64), disorder_hint=hint,
                                        features=features, plan=plan)
    return fetch(hc, labels, feats, k, offsets)


def batch_small(scale):
    chunks, dts, _ = hitgen.batch_64_chunks(scale=scale)
    return chunks, dts


def test_batch_64_chunks_scaled(hc):
    chunks, dts = batch_small(0.02)
    got, k = run(hc, chunks, dts, hint=512)
    compare(got, k, expect(chunks, dts), "batch x0.02")


def test_batch_uneven_sizes_and_tile_edges(hc):
    sizes = [1, 0, 2047, 2048, 2049, 8191, 8192, 8193, 0, 1023, 1025, 30000, 3, 70001, 0]
    chunks = [hitgen.blob_stream(m, 1000 + c, span_ticks=max(1, m * 64)) for c, m in enumerate(sizes)]
    dts = [(64, 128, 320)[c % 3] for c in range(len(sizes))]
    got, k = run(hc, chunks, dts, hint=512)
    compare(got, k, expect(chunks, dts), "uneven")


def test_batch_mixed_and_special_dts(hc):
    chunks = [hitgen.mixed_stream(200_000, 7, span_ticks=12_800_000),
              hitgen.uniform_hits(5000, 8, width=8, height=8, toa_hi=64),
              hitgen.blob_stream(40_000, 9, span_ticks=2_000_000),
              hitgen.blob_stream(40_000, 10, span_ticks=2_000_000),
              hitgen.mixed_stream(300_000, 11, span_ticks=19_200_000)]
    dts = [128, 3, oracle.DT_INFINITE, 0, 128]
    got, k = run(hc, chunks, dts, hint=4096)
    compare(got, k, expect(chunks, dts), "mixed")


def test_batch_single_chunk_and_labels_only(hc):
    chunks = [hitgen.mixed_stream(250_000, 21, span_ticks=16_000_000)]
    dts = [128]
    got, k = run(hc, chunks, dts, hint=4096)
    compare(got, k, expect(chunks, dts), "single")
    chunks2 = [hitgen.blob_stream(m, 30 + m, span_ticks=m * 64) for m in (5000, 17, 60000)]
    got, k = run(hc, chunks2, [128] * 3, hint=512, features=False)
    compare(got, k, expect(chunks2, [128] * 3), "labels-only")


def test_batch_all_empty(hc):
    got, k = run(hc, [np.empty(0, dtype=hitgen.HIT_DTYPE)] * 3, [128] * 3)
    assert list(k) == [0, 0, 0]


def test_batch_wide_chunk_and_range_error(hc):
    a = hitgen.blob_stream(1000, 41, span_ticks=64_000)
    b = hitgen.blob_stream(1000, 42, span_ticks=64_000)
    # a chunk whose ToA span needs 63 bits: sorted by the fallback beside a
    # 1-bit chunk field, still exact
    b["toa"][5] = np.uint64(1 << 63) + np.uint64(7)
    assert int(b["toa"].max()) - int(b["toa"].min()) < 1 << 63
    got, k = run(hc, [a, b], [128, 128], hint=512)
    compare(got, k, expect([a, b], [128, 128]), "wide chunk")
    # a span of 2^64 - 1 ticks leaves no room for the chunk field
    b["toa"][6] = np.uint64(0)
    b["toa"][5] = np.uint64((1 << 64) - 1)
    got, k = run(hc, [a, b], [128, 128], hint=512)
    assert list(k) == [hc.HC_ERR_RANGE, hc.HC_ERR_RANGE]


def test_batch_autotune_plan(hc):
    import torch
    chunks, dts = batch_small(0.01)
    hits, offsets = pack(chunks)
    d = hc.hits_to_device(hits)
    n = hits.size
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    feats = torch.empty((n, 64), dtype=torch.uint8, device="cuda")
    k = torch.empty(len(chunks), dtype=torch.int32, device="cuda")
    dts = np.asarray(dts, dtype=np.uint64)
    plan = hc.hc_batch_autotune(d, offsets, dts, labels, feats, k, disorder_hint=512)
    desc = plan.describe()
    print("plan:", desc, flush=True)
    assert "xcd_map=" in desc and "sort_tile=" in desc
    want = expect(chunks, dts)
    got, kk = fetch(hc, labels, feats, k, offsets)
    compare(got, kk, want, "autotune result")
    labels.fill_(-9)
    feats.fill_(0xAB)
    hc.hc_cluster_batch(d, offsets, dts, labels, feats, k, plan=plan)
    got, kk = fetch(hc, labels, feats, k, offsets)
    compare(got, kk, want, "with plan")
    plan.close()


def test_batch_graph_replays(hc):
    import torch
    chunks, dts = batch_small(0.01)
    hits, offsets = pack(chunks)
    alt = [hitgen.blob_stream(c.size, 500 + i, span_ticks=max(1, c.size * 64)) for i, c in enumerate(chunks)]
    hits_alt, _ = pack(alt)
    dts = np.asarray(dts, dtype=np.uint64)
    n = hits.size
    d = hc.hits_to_device(hits)
    labels = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    feats = torch.zeros((n, 64), dtype=torch.uint8, device="cuda")
    k = torch.empty(len(chunks), dtype=torch.int32, device="cuda")
    g = hc.hc_batch_graph_create(d, offsets, dts, labels, feats, k, disorder_hint=512)
    want = expect(chunks, dts)
    want_alt = expect(alt, dts)
    stream = torch.cuda.current_stream()
    for rep in range(4):
        src = hits_alt if rep % 2 else hits
        print("graph replay %d" % rep, flush=True)
        d.copy_(torch.from_numpy(src.view(np.uint8).reshape(-1)).cuda())
        labels.fill_(-9)
        feats.zero_()
        # eager work of the program's own between replays
        junk = torch.arange(1 << 20, device="cuda", dtype=torch.float32).sum()
        torch.cuda.synchronize()
        g.launch(stream)
        torch.cuda.synchronize()
        got, kk = fetch(hc, labels, feats, k, offsets)
        compare(got, kk, want_alt if rep % 2 else want, "replay %d" % rep)
        # the same batch eagerly, checked against the replay's output
        el, ef, ek = hc.cluster_batch(d, offsets, dts, disorder_hint=512)
        eg, ekk = fetch(hc, el, ef, ek, offsets)
        assert np.array_equal(ekk, kk)
        for (a, fa), (b, fb) in zip(eg, got):
            assert np.array_equal(a, b) and fa.tobytes() == fb.tobytes()
        del junk
    g.close()


def test_batch_64_chunks_full_size(hc):
    """The 64-chunk workload at its stated size (27.1M hits, chunks of 1k-2M
    hits, dt per chunk in {100, 200, 500} ns), default plan, every chunk
    element by element against the oracle."""
    from concurrent.futures import ThreadPoolExecutor
    chunks, dts, _ = hitgen.batch_64_chunks()
    got, k = run(hc, chunks, dts, hint=512)
    with ThreadPoolExecutor(8) as ex:
        want = list(ex.map(lambda cd: oracle.cluster(cd[0], 256, 256, int(cd[1])), zip(chunks, dts)))
    compare(got, k, want, "batch full size")


def test_batch_dense_shower_chunks(hc):
    """Chunks with dense showers: wide and deep link tiles inside a batch,
    whose halos must stop at their chunk's first hit."""
    chunks = [hitgen.shower_stream(m, hitgen.BASE_SEED + 70 + c, shower_hits=sh)
              for c, (m, sh) in enumerate([(150_000, (1500, 6000)), (3_000, (1100, 2000)), (200_000, (9000, 14000)),
                                           (90_000, (2500, 4000))])]
    dts = [128, 64, 128, 320]
    got, k = run(hc, chunks, dts, hint=4096)
    compare(got, k, expect(chunks, dts), "showers")
