"""GPU parity of the stream form: chunked pushes with exact stitching must
give the whole-stream oracle's labels and features, bit for bit."""
import numpy as np
import pytest

import hitgen
import oracle

pytestmark = pytest.mark.gpu

DT_STREAM = 128


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2412_11809_amd as hc
    assert torch.cuda.is_available()
    hc.load_library()
    return hc


def run_stream(hc, hits, sizes, w, h, dt, tdis, hint):
    import torch
    print("stream case: n=%d chunks=%d %dx%d dt=%d t=%d" % (hits.size, len(sizes), w, h, dt, tdis), flush=True)
    st = hc.HcStream(dt, tdis, w, h, hint)
    labels_dev = []
    done, feats = [], []
    at = 0
    for c, m in enumerate(sizes):
        d = hc.hits_to_device(hits[at:at + m])
        lab = torch.full((max(m, 1),), -7, dtype=torch.int32, device="cuda")
        st.push(d, lab, c)
        labels_dev.append((d, lab, m))
        tg, ft = st.poll()
        done += tg
        feats.append(ft)
        at += m
    st.flush()
    tg, ft = st.poll()
    done += tg
    feats.append(ft)
    torch.cuda.synchronize()
    labels = np.concatenate([lab[:m].cpu().numpy() for _, lab, m in labels_dev]) if sizes else np.empty(0, np.int32)
    feats = np.concatenate(feats)
    st.close()
    return labels, feats, done


def check(hc, hits, sizes, w, h, dt, hint, t_scale=1):
    tdis = (hitgen.realised_disorder_ticks(hits) + 1) * t_scale
    got_l, got_f, done = run_stream(hc, hits, sizes, w, h, dt, tdis, hint)
    want_l, want_f = oracle.cluster(hits, w, h, dt)
    assert sorted(done) == list(range(len(sizes)))
    bad = np.nonzero(got_l != want_l)[0]
    assert bad.size == 0, "%d labels differ, first %s: %s vs %s" % (bad.size, bad[:5], got_l[bad[:5]], want_l[bad[:5]])
    got_f = got_f[np.argsort(got_f["label"], kind="stable")]
    assert got_f.size == want_f.size
    assert got_f.tobytes() == want_f.tobytes()


def test_stream_timepix4_chunks(hc):
    hits, p = hitgen.timepix4_200m(n=3_000_000)
    check(hc, hits, [200_000] * 15, p["width"], p["height"], p["dt"], p["disorder"])


def test_stream_random_chunking(hc):
    hits, p = hitgen.blobs_100k(n=60_000, seed=77)
    rng = np.random.default_rng(5)
    sizes = []
    left = hits.size
    while left:
        m = int(min(left, rng.choice([1, 2, 7, 64, 1000, 5000])))
        sizes.append(m)
        left -= m
    check(hc, hits, sizes, 256, 256, p["dt"], p["disorder"])


def test_stream_mixed_workload(hc):
    hits, p = hitgen.mixed_10m(n=2_000_000, seed=8)
    check(hc, hits, [250_000] * 8, 256, 256, p["dt"], p["disorder"])


def test_stream_rejects_disorder_and_continues(hc):
    import torch
    hits, p = hitgen.blobs_100k(n=40_000, seed=9)
    tdis = hitgen.realised_disorder_ticks(hits) + 1
    st = hc.HcStream(p["dt"], tdis, 256, 256, p["disorder"])
    a, b = hits[:20_000], hits[20_000:]
    la = torch.empty(a.size, dtype=torch.int32, device="cuda")
    st.push(hc.hits_to_device(a), la, 0)
    bad = b[:100].copy()
    bad["toa"][50] = 0  # far below the watermark
    lbad = torch.full((bad.size,), -5, dtype=torch.int32, device="cuda")
    st.push(hc.hits_to_device(bad), lbad, 99)  # rejected on the device; reported by poll
    lb = torch.empty(b.size, dtype=torch.int32, device="cuda")
    st.push(hc.hits_to_device(b), lb, 1)
    st.flush()
    done, _ = st.poll()
    assert sorted(done) == [0, 1]
    assert st.rejected == {99: hc.HC_ERR_DISORDER}
    assert (lbad.cpu().numpy() == -5).all()
    got = np.concatenate([la.cpu().numpy(), lb.cpu().numpy()])
    want, _ = oracle.cluster(hits, 256, 256, p["dt"])
    assert (got == want).all()
    st.close()


def test_stream_timepix4_1m_chunks(hc):
    """The Timepix4-shaped workload at its own chunk shape: 16 consecutive
    1M-hit pushes of the 300 Mhit/s stream (448x512, displacement <= 16384),
    element by element against the whole-stream oracle."""
    n = 16_000_000
    hits = np.concatenate(list(hitgen.timepix4_stream(n=n, seed=hitgen.BASE_SEED + 14)))
    p = hitgen.TPX4_PARAMS
    check(hc, hits, [1_000_000] * 16, p["width"], p["height"], p["dt"], p["disorder"])


def test_stream_dense_shower_chunks(hc):
    # showers of 9000-14000 hits within 100 ns: link tiles whose halo exceeds
    # the wide kernel's go to the fallback, inside pushes whose open hits
    # ride ahead of each chunk
    hits = hitgen.shower_stream(900_000, seed=hitgen.BASE_SEED + 88, shower_hits=(9000, 14000))
    check(hc, hits, [150_000] * 6, 256, 256, DT_STREAM, 4096)


def test_stream_large_disorder_bound(hc):
    """A declared disorder bound ten times the realised one keeps about ten
    times more hits open (about 200k ahead of every 1M-hit chunk): the sort
    of open hits + chunk then reaches across dozens of tiles, and the result
    is still the whole-stream oracle's."""
    n = 8_000_000
    hits = np.concatenate(list(hitgen.timepix4_stream(n=n, seed=hitgen.BASE_SEED + 15)))
    p = hitgen.TPX4_PARAMS
    check(hc, hits, [1_000_000] * 8, p["width"], p["height"], p["dt"], p["disorder"], t_scale=10)


def _push_expect(hc, st, hits, tag):
    import torch
    lab = torch.full((hits.size,), -7, dtype=torch.int32, device="cuda")
    st.push(hc.hits_to_device(hits), lab, tag)
    return lab


def test_stream_no_watermark_while_max_below_t(hc):
    """While the largest ToA is still below the disorder bound t there is no
    watermark: a later hit at ToA 0 is valid (the t-ordered condition
    toa_i < toa_j + t holds for it) and nothing closes early."""
    a = hitgen.uniform_hits(300, 1, width=16, height=16, toa_hi=500)
    b = hitgen.uniform_hits(300, 2, width=16, height=16, toa_hi=500)
    b["toa"][:5] = 0
    hits = np.concatenate([a, b])
    tdis, dt = 1000, 3   # M stays below t throughout
    assert int(hits["toa"].max()) < tdis
    st = hc.HcStream(dt, tdis, 256, 256, 512)
    la = _push_expect(hc, st, a, 0)
    lb = _push_expect(hc, st, b, 1)
    done, _ = st.poll()
    assert done == []  # no watermark yet: nothing is final before the flush
    st.flush()
    done, feats = st.poll()
    assert sorted(done) == [0, 1]
    got = np.concatenate([la.cpu().numpy(), lb.cpu().numpy()])
    want_l, want_f = oracle.cluster(hits, 256, 256, dt)
    assert np.array_equal(got, want_l)
    feats = feats[np.argsort(feats["label"], kind="stable")]
    assert feats.tobytes() == want_f.tobytes()
    st.close()


def test_stream_push_after_flush(hc):
    """After a flush the stream continues as a new segment: a hit within dt
    of the largest flushed ToA is rejected (it could join a cluster whose
    labels are already final), a later chunk is accepted and clustered on its
    own."""
    a, p = hitgen.blobs_100k(n=30_000, seed=21)
    dt = p["dt"]
    tdis = hitgen.realised_disorder_ticks(a) + 1
    st = hc.HcStream(dt, tdis, 256, 256, p["disorder"])
    la = _push_expect(hc, st, a, 0)
    st.flush()
    M = int(a["toa"].max())
    late = a[:50].copy()
    late["toa"] = np.uint64(M + dt)     # exactly dt after the last flushed hit
    _push_expect(hc, st, late, 9)
    st.wait()
    done, _ = st.poll()
    assert st.rejected == {9: hc.HC_ERR_DISORDER}
    c = a.copy()
    c["toa"] += np.uint64(M + dt + 1 - int(a["toa"].min()))
    lc = _push_expect(hc, st, c, 1)
    st.flush()
    done += st.poll()[0]
    assert sorted(done) == [0, 1]
    want, _ = oracle.cluster(np.concatenate([a, c]), 256, 256, dt)
    got = np.concatenate([la.cpu().numpy(), lc.cpu().numpy()])
    assert np.array_equal(got, want)
    st.close()


def test_stream_push_chunks_equals_one_by_one(hc):
    """Several chunks per push give what pushing them one by one gives: the
    same labels, statuses and closed clusters, equal to the oracle over the
    accepted chunks.  Planted rejections: a chunk below every watermark, one
    off the sensor, and one that is late only against a chunk accepted
    earlier in the same push."""
    import torch
    base = hitgen.blob_stream(300_000, [hitgen.BASE_SEED + 9, 1], span_ticks=300_000 * 64, disorder=512)
    tdis = hitgen.realised_disorder_ticks(base) + 1
    rng = np.random.default_rng(19)
    chunks, at = [], 0
    while at < base.size:
        m = int(min(base.size - at, rng.integers(1, 24_000)))
        chunks.append(base[at:at + m])
        at += m
    assert len(chunks) > 20
    late = base[:500].copy()
    late["toa"] = 0
    off = base[1000:1200].copy()
    off["x"] = 300
    ref = len(chunks) // 3
    seq_late = chunks[ref][:1].copy()  # late against chunk `ref` only (same push below)
    seq_late["toa"] = int(chunks[ref]["toa"].max()) - tdis - 1
    assert int(seq_late["toa"][0]) > int(np.concatenate(chunks[:ref])["toa"].max()) - tdis
    chunks = chunks[:ref + 1] + [seq_late] + chunks[ref + 1:]
    mid = 2 * len(chunks) // 3
    chunks = chunks[:mid] + [late, off] + chunks[mid:]
    want_status = {ref + 1: hc.HC_ERR_DISORDER, mid: hc.HC_ERR_DISORDER, mid + 1: hc.HC_ERR_RANGE}
    # pushes of 1..16 chunks; `ref` and the chunk after it share one
    groups, j = [], 0
    while j < len(chunks):
        g = int(rng.integers(1, 17))
        if j <= ref < j + g <= ref + 1:
            g = ref + 2 - j
        groups.append(list(range(j, min(len(chunks), j + g))))
        j += g
    assert any(ref in g and ref + 1 in g for g in groups) and any(len(g) > 8 for g in groups)

    def serve(multi):
        st = hc.HcStream(DT_STREAM, tdis, 256, 256, 512)
        labs = [torch.full((c.size,), -7, dtype=torch.int32, device="cuda") for c in chunks]
        feats = []
        for g in (groups if multi else [[i] for i in range(len(chunks))]):
            d = hc.hits_to_device(np.concatenate([chunks[i] for i in g]))
            if multi:
                st.hc_stream_push_chunks(d, [chunks[i].size for i in g], [labs[i] for i in g], g)
            else:
                st.push(d, labs[g[0]], g[0])
            feats.append(st.poll()[1])
            torch.cuda.synchronize()  # d may go
        st.flush()
        feats.append(st.poll()[1])
        torch.cuda.synchronize()
        out = [lab.cpu().numpy() for lab in labs]
        rejected = dict(st.rejected)
        st.close()
        f = np.concatenate(feats)
        return out, rejected, f[np.argsort(f["label"], kind="stable")]

    one_l, one_r, one_f = serve(False)
    mul_l, mul_r, mul_f = serve(True)
    assert one_r == want_status and mul_r == want_status
    for i in range(len(chunks)):
        assert np.array_equal(one_l[i], mul_l[i]), "chunk %d" % i
    assert one_f.tobytes() == mul_f.tobytes()
    for i in want_status:
        assert (mul_l[i] == -7).all()
    kept = [i for i in range(len(chunks)) if i not in want_status]
    want_l, want_f = oracle.cluster(np.concatenate([chunks[i] for i in kept]), 256, 256, DT_STREAM)
    assert np.array_equal(np.concatenate([mul_l[i] for i in kept]), want_l)
    assert mul_f.tobytes() == want_f.tobytes()


def test_stream_push_chunks_argument_errors(hc):
    import torch
    st = hc.HcStream(DT_STREAM, 1 << 20, 256, 256, 512)
    d = torch.zeros(16 * 40, dtype=torch.uint8, device="cuda")
    lab = [torch.empty(20, dtype=torch.int32, device="cuda") for _ in range(17)]
    for counts in ([], [20] * 17, [20, 0]):
        with pytest.raises(hc.HcError) as ei:
            st.hc_stream_push_chunks(d, counts, lab[:len(counts)], list(range(len(counts))))
        assert ei.value.code == hc.HC_ERR_ARG
    # a stream that takes ids takes them with every push: several chunks at once carry none
    hits = hc.hits_to_device(hitgen.blob_stream(40, hitgen.BASE_SEED + 3, span_ticks=40 * 64, disorder=0))
    ids = torch.arange(40, dtype=torch.int32, device="cuda")
    lab40 = torch.empty(40, dtype=torch.int32, device="cuda")
    st.hc_stream_push_ids(hits, ids, 40, lab40, 0)
    with pytest.raises(hc.HcError) as ei:
        st.hc_stream_push_chunks(hits, [20, 20], lab[1:3], [1, 2])
    assert ei.value.code == hc.HC_ERR_ARG
    st.close()
