"""GPU parity of the stream form: chunked pushes with exact stitching must
give the whole-stream oracle's labels and features, bit for bit."""
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


def check(hc, hits, sizes, w, h, dt, hint):
    tdis = hitgen.realised_disorder_ticks(hits) + 1
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
    lbad = torch.empty(bad.size, dtype=torch.int32, device="cuda")
    with pytest.raises(hc.HcError) as e:
        st.push(hc.hits_to_device(bad), lbad, 99)
    assert e.value.code == hc.HC_ERR_DISORDER
    lb = torch.empty(b.size, dtype=torch.int32, device="cuda")
    st.push(hc.hits_to_device(b), lb, 1)
    st.flush()
    done, _ = st.poll()
    assert sorted(done) == [0, 1]
    got = np.concatenate([la.cpu().numpy(), lb.cpu().numpy()])
    want, _ = oracle.cluster(hits, 256, 256, p["dt"])
    assert (got == want).all()
    st.close()
