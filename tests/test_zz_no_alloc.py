"""hc_cluster_noalloc, called through the C-ABI, gives exactly what
hc_cluster gives (labels, feature rows, cluster count) on the same input:
two calls in a row, the second with a smaller input, so the second runs on
what the first left in the shared scratch array.  Also checked against the
oracle, and the size limit is refused before any device work."""
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


def outputs(hc, entry, d_hits, n, p, features=True):
    import torch
    dev = d_hits.device
    labels = torch.full((max(n, 1),), -7, dtype=torch.int32, device=dev)
    feats = torch.zeros((max(n, 1), 64), dtype=torch.uint8, device=dev) if features else None
    k = torch.full((1,), -9, dtype=torch.int32, device=dev)
    if entry == "noalloc":
        hc.hc_cluster_noalloc(d_hits, n, p["dt"], labels, feats, k, p["width"], p["height"], p["disorder"])
    else:
        hc.hc_cluster(d_hits, n, p["dt"], labels, feats, k, p["width"], p["height"], p["disorder"])
    torch.cuda.synchronize()
    kk = int(k.item())
    f = hc.features_to_numpy(feats, kk) if features else None
    return labels[:n].cpu().numpy(), f, kk


def compare(hc, hits, p, features=True):
    print("case: n=%d %dx%d dt=%d hint=%d features=%s" % (hits.size, p["width"], p["height"], p["dt"],
                                                           p["disorder"], features), flush=True)
    d = hc.hits_to_device(hits)
    n = hits.size
    got_l, got_f, got_k = outputs(hc, "noalloc", d, n, p, features)
    ref_l, ref_f, ref_k = outputs(hc, "plain", d, n, p, features)
    assert got_k == ref_k
    assert (got_l == ref_l).all()
    if features:
        assert got_f.tobytes() == ref_f.tobytes()
    return got_l, got_f, got_k


def test_two_calls_second_smaller(hc):
    hits, p = hitgen.mixed_10m(n=1_000_000, seed=4242)
    l1, f1, k1 = compare(hc, hits, p)
    want_l, want_f = oracle.cluster(hits, p["width"], p["height"], p["dt"])
    assert (l1 == want_l).all() and f1.tobytes() == want_f.tobytes() and k1 == want_f.size
    small, q = hitgen.blobs_100k(n=30_001, seed=77)
    l2, f2, k2 = compare(hc, small, q)
    want_l, want_f = oracle.cluster(small, q["width"], q["height"], q["dt"])
    assert (l2 == want_l).all() and f2.tobytes() == want_f.tobytes() and k2 == want_f.size


def test_labels_only_tail_and_empty(hc):
    import torch
    hits, p = hitgen.blobs_100k(n=4097, seed=5)
    compare(hc, hits, p, features=False)
    compare(hc, hits[:1], p)
    k = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    d = torch.empty(16, dtype=torch.uint8, device="cuda")
    hc.hc_cluster_noalloc(d, 0, 128, None, None, k)
    torch.cuda.synchronize()
    assert int(k.item()) == 0


def test_limit_refused_before_device_work(hc):
    import torch
    limit = hc.hc_noalloc_scratch_bytes()
    n = 1
    while hc.hc_workspace_size(n) <= limit:
        n *= 2
    d = torch.empty(16, dtype=torch.uint8, device="cuda")
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    # the size check comes before any pointer is used, so tiny buffers suffice
    with pytest.raises(hc.HcError) as e:
        hc.hc_cluster_noalloc(d, n, 128, d, None, k)
    assert e.value.code == hc.HC_ERR_WORKSPACE
    with pytest.raises(hc.HcError) as e:
        hc.hc_cluster_noalloc(d, 1, 128, d, None, k, flags=hc.HC_FLAG_GLOBAL_TIME)
    assert e.value.code == hc.HC_ERR_ARG
