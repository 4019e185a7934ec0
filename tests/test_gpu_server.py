"""GPU tests of the served form: every stream's labels and closed-cluster
features equal the whole-stream oracle's, and are the same bit for bit when
the stream is served alone and when it is served in a mix with other streams
under a tight slot and memory budget."""
import numpy as np
import pytest

import hitgen
import oracle

pytestmark = pytest.mark.gpu

DT = 128


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2412_11809_amd as hc
    assert torch.cuda.is_available()
    hc.load_library()
    return hc


def make_streams(k, n, seed):
    streams = []
    for s in range(k):
        h = hitgen.blob_stream(n + 7919 * s, [seed, s], span_ticks=(n + 7919 * s) * 64, disorder=512)
        rng = np.random.default_rng([seed, s, 1])
        sizes = []
        left = h.size
        while left > 0:
            m = min(left, int(np.exp(rng.uniform(np.log(4000), np.log(64000)))))
            sizes.append(m)
            left -= m
        streams.append((h, sizes))
    return streams


def pinned_copy(a):
    import torch
    t = torch.empty(a.nbytes, dtype=torch.uint8, pin_memory=True)
    t.numpy()[:] = a.view(np.uint8).reshape(-1)
    return t


def serve(hc, streams, ids, max_slots, budget, max_chunk=65536):
    """Submit the chunks of streams[ids] interleaved by chunk position; returns
    per stream (labels, closed features sorted by label) and the stats."""
    import torch
    tdis = max(hitgen.realised_disorder_ticks(streams[i][0]) for i in ids) + 1
    srv = hc.HcServer(len(ids), DT, tdis, max_slots=max_slots, hbm_budget=budget, disorder_hint=512,
                      max_chunk_hits=max_chunk)
    labels = {}
    plan = []
    for j, i in enumerate(ids):
        h, sizes = streams[i]
        labels[i] = torch.full((h.size,), -5, dtype=torch.int32, pin_memory=True)
        at = 0
        for c, m in enumerate(sizes):
            plan.append((c, j, i, at, m))
            at += m
    plan.sort()
    completions = []
    for c, j, i, at, m in plan:
        h = streams[i][0]
        hits = pinned_copy(h[at:at + m])
        srv.submit(j, hits, labels[i][at:at + m], tag=c)
        completions.append(srv.poll())
    for j in range(len(ids)):
        srv.flush(j)
    srv.wait_idle(120000)
    completions.append(srv.poll())
    comp = np.concatenate(completions)
    stats = srv.stats()
    out = {}
    for j, i in enumerate(ids):
        f = srv.closed(j)
        out[i] = (labels[i].numpy().copy(), f[np.argsort(f["label"], kind="stable")])
    srv.close()
    return out, comp, stats


def test_server_alone_equals_mix_equals_oracle(hc):
    streams = make_streams(4, 150_000, hitgen.BASE_SEED + 5)
    print("server: alone", flush=True)
    alone, comp_a, st_a = serve(hc, streams, [0], max_slots=1, budget=0)
    print("server: mix", flush=True)
    mix, comp_m, st_m = serve(hc, streams, [0, 1, 2, 3], max_slots=2, budget=320 << 20)
    print("stats alone", st_a, "\nstats mix", st_m, flush=True)
    assert (comp_a["status"] == 0).all() and (comp_m["status"] == 0).all()
    assert len(comp_m) == sum(len(s[1]) for s in streams)
    assert st_m["hbm_peak"] <= 320 << 20
    assert 1 <= st_m["peak_slots_in_use"] <= 2
    assert st_m["processing_p50"] <= st_m["processing_p99"]
    assert st_m["final_p50"] <= st_m["final_p99"]
    # alone == mix, bit for bit
    la, fa = alone[0]
    lm, fm = mix[0]
    assert np.array_equal(la, lm)
    assert fa.tobytes() == fm.tobytes()
    # every stream == whole-stream oracle
    for i in range(4):
        h = streams[i][0]
        want_l, want_f = oracle.cluster(h, 256, 256, DT)
        got_l, got_f = mix[i]
        bad = np.nonzero(got_l != want_l)[0]
        assert bad.size == 0, "stream %d: %d labels differ" % (i, bad.size)
        assert got_f.tobytes() == want_f.tobytes(), "stream %d features differ" % i


def test_server_rejections(hc):
    import torch
    h = hitgen.blob_stream(20_000, hitgen.BASE_SEED + 6, span_ticks=20_000 * 64, disorder=64)
    tdis = hitgen.realised_disorder_ticks(h) + 1
    srv = hc.HcServer(1, DT, tdis, max_slots=1, hbm_budget=64 << 20, disorder_hint=512, max_chunk_hits=16384)
    # a chunk that can never fit the budget is refused at submit
    big = torch.empty(16 * (8 << 20), dtype=torch.uint8)
    lab_big = torch.empty(8 << 20, dtype=torch.int32)
    with pytest.raises(hc.HcError) as ei:
        srv.submit(0, big, lab_big, tag=99)
    assert ei.value.code == hc.HC_ERR_BUDGET
    lab = torch.full((h.size,), -5, dtype=torch.int32)
    srv.submit(0, h[:10_000].copy(), lab[:10_000], tag=0)
    # far in the past: below the watermark, rejected; the stream continues
    late = h[:100].copy()
    late["toa"] = 0
    lab_late = torch.full((100,), -5, dtype=torch.int32)
    srv.submit(0, late, lab_late, tag=1)
    srv.submit(0, h[10_000:].copy(), lab[10_000:], tag=2)
    srv.flush(0)
    srv.wait_idle(60000)
    comp = srv.poll()
    status = {int(c["tag"]): int(c["status"]) for c in comp}
    assert status == {0: 0, 1: hc.HC_ERR_DISORDER, 2: 0}
    assert (lab_late.numpy() == -5).all()
    want_l, want_f = oracle.cluster(h, 256, 256, DT)
    assert np.array_equal(lab.numpy(), want_l)
    f = srv.closed(0)
    f = f[np.argsort(f["label"], kind="stable")]
    assert f.tobytes() == want_f.tobytes()
    srv.close()


@pytest.mark.parametrize("read", ["while_serving", "into_small_buffer", "at_end"])
def test_server_closed_records_read_while_serving(hc, read):
    """A stream that closes about 333k clusters, its closed-cluster records
    read while it is served (whole, or through a small reused buffer that
    splits the server's blocks, whose read-out blocks it then reuses) or only
    at the end: every record arrives once and equals the oracle's, and the
    labels are the oracle's."""
    import torch
    n, m = 2_000_000, 100_000
    h = hitgen.blob_stream(n, [hitgen.BASE_SEED + 7, 0], span_ticks=n * 64, disorder=512)
    tdis = hitgen.realised_disorder_ticks(h) + 1
    srv = hc.HcServer(1, DT, tdis, disorder_hint=512, max_chunk_hits=m)
    lab = torch.full((n,), -5, dtype=torch.int32, pin_memory=True)
    hits = pinned_copy(h)
    got, comp = [], []
    buf = np.zeros(10_007, dtype=hc.FEATURE_DTYPE)

    def read_small():
        while True:
            k = srv.closed_into(0, buf)
            got.append(buf[:k].copy())
            if k < buf.size:
                return

    for c, at in enumerate(range(0, n, m)):
        srv.submit(0, hits[16 * at:16 * (at + m)], lab[at:at + m], tag=c)
        if read == "while_serving":
            got.append(srv.closed(0))
        elif read == "into_small_buffer":
            read_small()
        if read != "at_end":
            comp.append(srv.poll())
    srv.flush(0)
    srv.wait_idle(120000)
    comp.append(srv.poll())
    got.append(srv.closed(0))
    srv.close()
    comp = np.concatenate(comp)
    assert len(comp) == n // m and (comp["status"] == 0).all()
    want_l, want_f = oracle.cluster(h, 256, 256, DT)
    assert np.array_equal(lab.numpy(), want_l)
    f = np.concatenate(got)
    assert f.size == want_f.size
    f = f[np.argsort(f["label"], kind="stable")]
    assert f.tobytes() == want_f.tobytes()


def test_server_merges_queued_chunks(hc):
    """Small chunks queued behind a running push are merged into fewer pushes,
    each chunk still accepted or rejected on its own: a late chunk among them
    is rejected, every other chunk's labels and the closed clusters equal the
    oracle's over the accepted chunks."""
    import torch
    n = 400_000
    h = hitgen.blob_stream(n, [hitgen.BASE_SEED + 8, 0], span_ticks=n * 64, disorder=512)
    tdis = hitgen.realised_disorder_ticks(h) + 1
    srv = hc.HcServer(1, DT, tdis, max_slots=1, disorder_hint=512)
    hits = pinned_copy(h)
    lab = torch.full((n,), -5, dtype=torch.int32, pin_memory=True)
    late = h[:300].copy()
    late["toa"] = 0
    lab_late = torch.full((300,), -5, dtype=torch.int32, pin_memory=True)
    m, c = 5000, 0
    for at in range(0, n, m):
        srv.submit(0, hits[16 * at:16 * (at + m)], lab[at:at + m], tag=c)
        c += 1
        if c == 40:
            srv.submit(0, late, lab_late, tag=1000)
    srv.flush(0)
    srv.wait_idle(120000)
    comp = srv.poll()
    stats = srv.stats()
    f = srv.closed(0)
    srv.close()
    status = {int(x["tag"]): int(x["status"]) for x in comp}
    assert len(status) == n // m + 1 and status.pop(1000) == hc.HC_ERR_DISORDER
    assert set(status.values()) == {0}
    print("pushes %d for %d chunks" % (stats["pushes"], n // m + 1), flush=True)
    assert stats["pushes"] < n // m
    assert (lab_late.numpy() == -5).all()
    want_l, want_f = oracle.cluster(h, 256, 256, DT)
    assert np.array_equal(lab.numpy(), want_l)
    f = f[np.argsort(f["label"], kind="stable")]
    assert f.tobytes() == want_f.tobytes()
