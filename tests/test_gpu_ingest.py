"""GPU parity of the host ingest front end (hc_ingest_*): hits fed in
arrival order, in pieces of any size, are buffered by the paper's buffer
filling (late hits move to the next buffer), clustered on the device with
exact stitching, and every label -- the smallest arrival index of the
hit's cluster -- must equal the whole-stream oracle's."""
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


def run(hc, hits, w, h, dt, hint, b, bt, t_closing, pieces, n_buffers=0, seed=0):
    import torch
    t = hitgen.realised_disorder_ticks(hits) + 1
    print("ingest case: n=%d b=%d b_t=%d t=%d t_closing=%d" % (hits.size, b, bt, t, t_closing), flush=True)
    labels = torch.full((max(hits.size, 1),), -1, dtype=torch.int32, pin_memory=True)
    ing = hc.HcIngest(labels, dt, t, t_closing, b, bt, w, h, hint, n_buffers)
    rng = np.random.default_rng(seed)
    at = 0
    while at < hits.size:
        m = int(min(hits.size - at, rng.choice(pieces)))
        ing.feed(np.ascontiguousarray(hits[at:at + m]))
        at += m
    ing.finish()
    st = ing.stats()
    ing.close()
    return labels.numpy()[:hits.size].copy(), st


def check(hc, hits, w, h, dt, hint, **kw):
    got, st = run(hc, hits, w, h, dt, hint, **kw)
    want, _ = oracle.cluster(hits, w, h, dt, features=False)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%d labels differ, first %s: %s vs %s" % (bad.size, bad[:5], got[bad[:5]], want[bad[:5]])
    assert st["hits_done"] == hits.size == st["hits_fed"]
    print(st, flush=True)
    return st


def test_ingest_mixed_stream(hc):
    hits, p = hitgen.mixed_10m(n=2_000_000, seed=61)
    st = check(hc, hits, 256, 256, p["dt"], p["disorder"], b=300_000, bt=20_000, t_closing=40_000,
               pieces=[1, 100, 4096, 65536, 200_000])
    assert st["buffers_sent"] >= 6 and st["diverted"] > 0


def test_ingest_timepix4(hc):
    hits = np.concatenate(list(hitgen.timepix4_stream(n=3_000_000, seed=62)))
    q = hitgen.TPX4_PARAMS
    st = check(hc, hits, q["width"], q["height"], q["dt"], q["disorder"], b=1 << 20, bt=60_000, t_closing=2048,
               pieces=[65536, 1 << 20])
    assert st["diverted"] > 0


def test_ingest_small_buffers_and_three_slots(hc):
    hits, p = hitgen.blobs_100k(n=80_000, seed=63)
    st = check(hc, hits, 256, 256, p["dt"], p["disorder"], b=6000, bt=1500, t_closing=200, pieces=[7, 999, 5000],
               n_buffers=3)
    assert st["buffers_sent"] >= 14


def test_ingest_empty_and_tiny(hc):
    check(hc, np.empty(0, dtype=hitgen.HIT_DTYPE), 256, 256, 128, 512, b=100, bt=10, t_closing=10, pieces=[1])
    one = hitgen.blob_stream(3, 64, span_ticks=10)
    check(hc, one, 256, 256, 128, 512, b=100, bt=10, t_closing=10, pieces=[1])
