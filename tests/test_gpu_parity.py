"""GPU parity: labels and features of hc_cluster, called through the C-ABI,
must equal the oracle's bit for bit (integer labels and sums exactly; the
centroid doubles bit-exactly, as both sides perform one correctly rounded
IEEE division of the same exact integers)."""
import numpy as np
import pytest

import hitgen
import oracle
from refs import canonical, check_invariants

pytestmark = pytest.mark.gpu

U64MAX = (1 << 64) - 1


@pytest.fixture(scope="module")
def hc():
    import torch
    import paper_2412_11809_amd as hc
    assert torch.cuda.is_available()
    hc.load_library()
    return hc


def run_gpu(hc, hits, w, h, dt, hint=0, features=True, stream=None, workspace=None, flags=0):
    import torch
    print("case: n=%d %dx%d dt=%d hint=%d flags=%d" % (hits.size, w, h, dt, hint, flags), flush=True)
    d = hc.hits_to_device(hits)
    labels, feats, k = hc.cluster(d, dt, w, h, disorder_hint=hint, features=features, stream=stream,
                                  workspace=workspace, flags=flags)
    torch.cuda.synchronize()
    kk = int(k.item())
    return labels.cpu().numpy(), (hc.features_to_numpy(feats, kk) if features else None), kk


def assert_parity(hc, hits, w, h, dt, hint=0, flags=0):
    got_l, got_f, k = run_gpu(hc, hits, w, h, dt, hint, flags=flags)
    want_l, want_f = oracle.cluster(hits, w, h, dt)
    assert k == want_f.size, "cluster count %d, oracle %d" % (k, want_f.size)
    bad = np.nonzero(got_l != want_l)[0]
    assert bad.size == 0, "%d labels differ, first at %s: got %s want %s" % (
        bad.size, bad[:5], got_l[bad[:5]], want_l[bad[:5]])
    assert got_f.tobytes() == want_f.tobytes(), "features differ"
    return got_l


def test_blobs_100k_full(hc):
    hits, p = hitgen.blobs_100k()
    assert_parity(hc, hits, p["width"], p["height"], p["dt"], p["disorder"])


def test_mixed_slice(hc):
    hits, p = hitgen.mixed_10m(n=1_000_000, seed=99)
    assert_parity(hc, hits, p["width"], p["height"], p["dt"], p["disorder"])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1023, 1024, 1025, 2047, 2048, 2049, 4097,
                               8191, 8192, 8193, 65535, 65537, 200_003])
def test_sizes(hc, n):
    hits = hitgen.blob_stream(n, [5, n], span_ticks=max(64, n * 64), disorder=512)
    assert_parity(hc, hits, 256, 256, 128, 512)


def test_empty(hc):
    import torch
    import paper_2412_11809_amd as m
    d = torch.empty(16, dtype=torch.uint8, device="cuda")
    labels = torch.empty(1, dtype=torch.int32, device="cuda")
    k = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    m.hc_cluster(d, 0, 10, labels, None, k)
    torch.cuda.synchronize()
    assert k.item() == 0


@pytest.mark.parametrize("hint", [0, 64, 512, 4096, 16384, 1 << 20])
def test_disorder_hints(hc, hint):
    """A wrong hint may cost speed, never exactness."""
    hits = hitgen.blob_stream(300_000, [6, hint], disorder=6000, span_ticks=300_000 * 64)
    assert_parity(hc, hits, 256, 256, 128, hint)


def test_reversed_input(hc):
    hits, p = hitgen.blobs_100k(n=50_000, seed=3)
    hits = hits[np.argsort(hits["toa"], kind="stable")][::-1].copy()
    assert_parity(hc, hits, 256, 256, p["dt"], 512)


def test_dt_infinite_is_image_labelling(hc):
    hits = hitgen.uniform_hits(40_000, 8, 256, 256, 1 << 30)
    assert_parity(hc, hits, 256, 256, U64MAX, 512)


def test_dt_zero(hc):
    hits = hitgen.uniform_hits(60_000, 9, 64, 64, 5000, disorder=100)
    assert_parity(hc, hits, 64, 64, 0, 128)


def test_single_pixel(hc):
    rng = np.random.default_rng(10)
    hits = np.zeros(30_000, dtype=oracle.HIT_DTYPE)
    hits["x"], hits["y"] = 17, 200
    hits["toa"] = np.sort(rng.integers(0, 3_000_000, hits.size))
    hits["tot"] = rng.integers(0, 50, hits.size)
    assert_parity(hc, hits, 256, 256, 128, 512)


def test_all_same_toa(hc):
    hits = hitgen.uniform_hits(20_000, 11, 100, 100, 1)
    assert_parity(hc, hits, 100, 100, 5, 512)


def test_wide_toa_range(hc):
    rng = np.random.default_rng(12)
    hits = hitgen.uniform_hits(50_000, 12, 256, 256, 1)
    hits["toa"] = np.sort(rng.integers(0, 1 << 62, hits.size)).astype(np.uint64)
    hits["toa"][::7] += np.uint64(3)  # near-ties
    assert_parity(hc, hits, 256, 256, 1 << 40, 512)


def test_dense_small_sensor(hc):
    hits = hitgen.uniform_hits(100_000, 13, 8, 8, 2_000_000, disorder=50)
    assert_parity(hc, hits, 8, 8, 30, 64)


def test_timepix4_sensor(hc):
    hits, p = hitgen.timepix4_200m(n=2_000_000)
    assert_parity(hc, hits, p["width"], p["height"], p["dt"], p["disorder"])


def test_edges_of_sensor(hc):
    rng = np.random.default_rng(14)
    n = 50_000
    hits = np.zeros(n, dtype=oracle.HIT_DTYPE)
    hits["x"] = rng.choice([0, 1, 254, 255], n)
    hits["y"] = rng.choice([0, 1, 254, 255], n)
    hits["toa"] = np.sort(rng.integers(0, 50_000, n))
    hits["tot"] = rng.integers(0, 1000, n)
    assert_parity(hc, hits, 256, 256, 3, 512)


def test_range_error_reported(hc):
    hits, p = hitgen.blobs_100k(n=10_000, seed=4)
    hits["x"][1234] = 256
    _, _, k = run_gpu(hc, hits, 256, 256, 128, 512)
    assert k == hc.HC_ERR_RANGE


def test_repeatable(hc):
    """Labels are schedule-independent: 20 repetitions agree exactly."""
    hits, p = hitgen.mixed_10m(n=400_000, seed=21)
    want = assert_parity(hc, hits, 256, 256, p["dt"], p["disorder"])
    for _ in range(20):
        got, _, _ = run_gpu(hc, hits, 256, 256, p["dt"], p["disorder"])
        assert (got == want).all()


def test_side_stream_and_workspace(hc):
    import torch
    hits, p = hitgen.blobs_100k(n=70_000, seed=5)
    ws = torch.empty(hc.hc_workspace_size(hits.size, 256, 256, 512), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    got, gf, k = run_gpu(hc, hits, 256, 256, p["dt"], 512, stream=s, workspace=ws)
    want, wf = oracle.cluster(hits, 256, 256, p["dt"])
    assert (got == want).all() and gf.tobytes() == wf.tobytes()


def test_small_workspace_rejected(hc):
    import torch
    d = hc.hits_to_device(hitgen.blobs_100k(n=5000)[0])
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    labels = torch.empty(5000, dtype=torch.int32, device="cuda")
    k = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(hc.HcError) as e:
        hc.hc_cluster(d, 5000, 128, labels, None, k, workspace=ws)
    assert e.value.code == hc.HC_ERR_WORKSPACE


def test_labels_only(hc):
    hits, p = hitgen.blobs_100k(n=30_000, seed=6)
    got, _, k = run_gpu(hc, hits, 256, 256, p["dt"], 512, features=False)
    want, wf = oracle.cluster(hits, 256, 256, p["dt"])
    assert (got == want).all() and k == wf.size


def test_mixed_10m_full_size(hc):
    """The benchmark's workload (10M hits) in the benchmark's configuration."""
    hits, p = hitgen.mixed_10m()
    got = assert_parity(hc, hits, p["width"], p["height"], p["dt"], p["disorder"])
    assert (got <= np.arange(got.size)).all()


# ---- dense showers: tiles with more than 1024 hits within dt before them go
# to the wide second level (halo up to 7168 hits), deeper ones on to the
# fallback over their windows; both search variants, and a batch of shower chunks
@pytest.mark.parametrize("showers", [(1500, 6000), (9000, 14000)])
@pytest.mark.parametrize("flags", [0, 2])
def test_dense_showers(hc, showers, flags):
    hits = hitgen.shower_stream(600_000, seed=hitgen.BASE_SEED + 40 + showers[0], shower_hits=showers)
    assert_parity(hc, hits, 256, 256, 128, 4096, flags=flags)


def test_dense_showers_timepix4_sensor(hc):
    hits = hitgen.shower_stream(500_000, seed=hitgen.BASE_SEED + 47, width=448, height=512,
                                shower_hits=(2000, 7000), radius=60)
    assert_parity(hc, hits, 448, 512, 1024, 4096)


# ---- each neighbour search forced on every tile (pixel index, window scan),
# and sensors at and beyond the window scan's 14-bit limit
@pytest.mark.parametrize("case", ["blobs_100k", "mixed_10m", "single_pixel", "dense", "timepix4", "same_toa"])
@pytest.mark.parametrize("variant", ["index", "window"])
def test_link_variants(hc, case, variant):
    flag = hc.HC_FLAG_LINK_PIXEL_INDEX if variant == "index" else hc.HC_FLAG_LINK_WINDOW
    if case == "blobs_100k":
        hits, p = hitgen.blobs_100k()
        assert_parity(hc, hits, 256, 256, p["dt"], p["disorder"], flags=flag)
    elif case == "mixed_10m":
        hits, p = hitgen.mixed_10m(n=1_000_000, seed=98)
        assert_parity(hc, hits, 256, 256, p["dt"], p["disorder"], flags=flag)
    elif case == "single_pixel":
        rng = np.random.default_rng(20)
        hits = np.zeros(30_000, dtype=oracle.HIT_DTYPE)
        hits["x"], hits["y"] = 255, 0
        hits["toa"] = np.sort(rng.integers(0, 3_000_000, hits.size))
        assert_parity(hc, hits, 256, 256, 128, 512, flags=flag)
    elif case == "dense":
        hits = hitgen.uniform_hits(100_000, 21, 8, 8, 2_000_000, disorder=50)
        assert_parity(hc, hits, 8, 8, 30, 64, flags=flag)
    elif case == "timepix4":
        hits, p = hitgen.timepix4_200m(n=1_000_000, seed=22)
        assert_parity(hc, hits, p["width"], p["height"], p["dt"], p["disorder"], flags=flag)
    else:
        hits = hitgen.uniform_hits(20_000, 23, 100, 100, 1)
        assert_parity(hc, hits, 100, 100, 5, 512, flags=flag)


def test_zero_tot_regions(hc):
    # clusters left of x = 128 have ToT 0 throughout (their centroid is the
    # unweighted mean), clusters across x = 128 mix zero and non-zero ToT
    hits, p = hitgen.mixed_10m(n=300_000, seed=97)
    hits["tot"][hits["x"] < 128] = 0
    assert_parity(hc, hits, p["width"], p["height"], p["dt"], p["disorder"])


@pytest.mark.parametrize("w,h", [(16384, 8), (8, 16384), (16385, 3), (3, 40000)])
def test_large_sensor_coordinates(hc, w, h):
    # clusters at the far corners: window scan up to 16384, pixel index beyond
    rng = np.random.default_rng(w + h)
    n = 40_000
    hits = np.zeros(n, dtype=oracle.HIT_DTYPE)
    cx = rng.choice([0, 1, w - 2, w - 1], n)
    cy = rng.choice([0, 1, h - 2, h - 1], n)
    hits["x"], hits["y"] = cx, cy
    hits["toa"] = np.sort(rng.integers(0, 4_000_000, n))
    hits["tot"] = rng.integers(1, 100, n)
    assert_parity(hc, hits, w, h, 100, 512)


@pytest.mark.parametrize("w,h", [(20000, 24), (600, 600)])
def test_sensor_beyond_both_searches(hc, w, h):
    # wider than the window scan's 14-bit limit and too many pixels for the
    # LDS bitmap (or, for 600 x 600, the index forced on a sensor too large
    # for it): every link tile goes to the link fallback, whose windows
    # then cover the whole input
    rng = np.random.default_rng(w * h)
    n = 60_000
    hits = np.zeros(n, dtype=oracle.HIT_DTYPE)
    hits["x"] = rng.choice([0, 1, 2, w // 2, w - 2, w - 1], n)
    hits["y"] = rng.choice([0, 1, h // 2, h - 2, h - 1], n)
    hits["toa"] = np.sort(rng.integers(0, 3_000_000, n))
    hits["tot"] = rng.integers(1, 100, n)
    flags = hc.HC_FLAG_LINK_PIXEL_INDEX if w < 16384 else 0
    assert_parity(hc, hits, w, h, 100, 512, flags=flags)


def test_random_sweep(hc):
    """300 seeded random configurations: stream kind, size (log-uniform
    50..200k), sensor, dt, disorder hint and neighbour-search variant."""
    rng = np.random.default_rng(2412)
    for case in range(300):
        kind = ["blobs", "mixed", "uniform", "tpx4"][int(rng.integers(4))]
        n = int(np.exp(rng.uniform(np.log(50), np.log(200_000))))
        seed = int(rng.integers(1 << 30))
        if kind == "blobs":
            hits = hitgen.blob_stream(n, seed, 256, 256, span_ticks=max(64, n * int(rng.choice([8, 64, 640]))),
                                      disorder=int(rng.choice([0, 64, 512, 4096])))
            w = h = 256
            dt = int(rng.choice([1, 32, 128, 1000]))
        elif kind == "mixed":
            hits, _ = hitgen.mixed_10m(n=n, seed=seed)
            w = h = 256
            dt = int(rng.choice([64, 128, 400]))
        elif kind == "uniform":
            w, h = int(rng.integers(1, 40)), int(rng.integers(1, 40))
            hits = hitgen.uniform_hits(n, seed, w, h, n * int(rng.choice([1, 10, 100])) + 1,
                                       disorder=int(rng.choice([0, 30, 300])))
            dt = int(rng.choice([0, 5, 50]))
        else:
            hits, p = hitgen.timepix4_200m(n=n, seed=seed)
            w, h, dt = p["width"], p["height"], p["dt"]
        hint = int(rng.choice([0, 256, 1024, 4096, 16384]))
        flags = int(rng.choice([0, hc.HC_FLAG_LINK_PIXEL_INDEX, hc.HC_FLAG_LINK_WINDOW]))
        print("sweep case", case, kind, n, seed, flush=True)
        assert_parity(hc, hits, w, h, dt, hint, flags=flags)
