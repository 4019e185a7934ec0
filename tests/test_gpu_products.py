"""GPU parity of the per-cluster products (hc_cluster_products, through the
C ABI): bounding boxes, filtered rows and the cluster-major grouping of the
kept hits must equal the product oracle's element by element, on top of
hc_cluster's own output."""
import numpy as np
import pytest

import hitgen
import oracle
from oracle import products

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2412_11809_amd as hc
    assert torch.cuda.is_available()
    hc.load_library()
    return hc


def run(hc, hits, w, h, dt, hint, flt):
    import torch
    n = hits.size
    print("products case: n=%d filter=%s" % (n, flt), flush=True)
    cap = max(n, 1)
    d = hc.hits_to_device(hits) if n else torch.empty(16, dtype=torch.uint8, device="cuda")
    labels = torch.empty(cap, dtype=torch.int32, device="cuda")
    feats = torch.empty((cap, 64), dtype=torch.uint8, device="cuda")
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    hc.hc_cluster(d, n, dt, labels, feats, k, w, h, hint)
    boxes = torch.full((cap, 8), 0xEE, dtype=torch.uint8, device="cuda")
    keep = torch.full((cap,), -3, dtype=torch.int32, device="cuda")
    nkeep = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    grouped = torch.zeros((cap, 16), dtype=torch.uint8, device="cuda")
    gidx = torch.full((cap,), -4, dtype=torch.int32, device="cuda")
    start = torch.full((cap + 1,), -6, dtype=torch.int64, device="cuda")
    hc.hc_cluster_products(d, n, labels, feats, k, keep, nkeep, boxes=boxes, grouped=grouped, grouped_idx=gidx,
                           row_start=start, filter=flt)
    torch.cuda.synchronize()
    K, nk = int(k.item()), int(nkeep.item())
    return (K, boxes[:K].cpu().numpy().reshape(-1).view(hc.BOX_DTYPE), keep[:max(nk, 0)].cpu().numpy(), nk,
            grouped.cpu().numpy().reshape(-1).view(hc.HIT_DTYPE), gidx.cpu().numpy(), start.cpu().numpy())


def check(hc, hits, w, h, dt, hint=0, flt=None):
    K, boxes, keep, nk, grouped, gidx, start = run(hc, hits, w, h, dt, hint, flt)
    labels, feats = oracle.cluster(hits, w, h, dt)
    assert K == feats.size
    assert boxes.tobytes() == products.boxes(hits, labels, feats).tobytes()
    rows = products.keep_rows(feats, **(flt or {}))
    assert nk == rows.size
    assert np.array_equal(keep, rows)
    idx, at = products.grouped(labels, feats, rows)
    m = idx.size
    assert np.array_equal(gidx[:m], idx)
    assert (gidx[m:] == -4).all()  # nothing written beyond the kept hits
    assert grouped[:m].tobytes() == hits[idx].tobytes()
    assert np.array_equal(start[:rows.size + 1], at)


def test_products_mixed(hc):
    hits, p = hitgen.mixed_10m(n=1_000_000, seed=31)
    check(hc, hits, 256, 256, p["dt"], p["disorder"])


def test_products_filtered(hc):
    hits, p = hitgen.mixed_10m(n=600_000, seed=32)
    t0 = int(np.quantile(hits["toa"], 0.3))
    check(hc, hits, 256, 256, p["dt"], p["disorder"],
          dict(min_size=3, max_size=400, min_sum_tot=200, max_sum_tot=1 << 40, toa_from=t0))


def test_products_blobs_and_tpx4(hc):
    hits, p = hitgen.blobs_100k()
    check(hc, hits, 256, 256, p["dt"], p["disorder"], dict(max_size=5))
    hits = np.concatenate(list(hitgen.timepix4_stream(n=2_000_000, seed=33)))
    q = hitgen.TPX4_PARAMS
    check(hc, hits, q["width"], q["height"], q["dt"], q["disorder"], dict(min_size=2))


def test_products_edges(hc):
    check(hc, np.empty(0, dtype=hitgen.HIT_DTYPE), 256, 256, 128)
    one = np.zeros(1, dtype=hitgen.HIT_DTYPE)
    one["x"], one["y"] = 255, 0
    check(hc, one, 256, 256, 128)
    hits, p = hitgen.blobs_100k(n=50_000, seed=34)
    check(hc, hits, 256, 256, p["dt"], p["disorder"], dict(min_size=10 ** 6))  # keeps nothing
    dense = hitgen.uniform_hits(70_001, 35, width=8, height=8, toa_hi=5000)
    check(hc, dense, 8, 8, 3, 0, dict(min_size=1))
