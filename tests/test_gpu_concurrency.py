"""Calls on different HIP streams are independent, also when both leave the
workspace to the library: two host threads, each on its own stream, run
hc_cluster and hc_cluster_batch with a NULL workspace at the same time (sizes
chosen so that the second round grows the cached buffers), and both results
are bit-exact against the oracle."""
import threading

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


def test_two_streams_null_workspace(hc):
    import torch
    plain = [hitgen.mixed_10m(n=m, seed=40 + m % 7)[0] for m in (300_000, 1_200_000)]
    batch = [[hitgen.blob_stream(m, [50, r, c], span_ticks=m * 64) for c, m in enumerate(sizes)]
             for r, sizes in enumerate(([20_000, 5_000, 90_000], [400_000, 7, 250_000, 60_000]))]
    want_plain = [oracle.cluster(h, 256, 256, 128) for h in plain]
    want_batch = [[oracle.cluster(c, 256, 256, 128) for c in b] for b in batch]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    out = {}
    errors = []
    start = threading.Barrier(2)

    def run_plain(r):
        try:
            with torch.cuda.stream(s1):
                d = hc.hits_to_device(plain[r])
                start.wait()
                for rep in range(3):
                    labels, feats, k = hc.cluster(d, 128, stream=s1)
                    s1.synchronize()
                    out[("plain", r, rep)] = (labels.cpu().numpy(), hc.features_to_numpy(feats, int(k.item())))
        except Exception as e:  # reported by the main thread
            errors.append(e)
            start.abort()

    def run_batch(r):
        try:
            with torch.cuda.stream(s2):
                hits = np.concatenate(batch[r])
                offsets = np.zeros(len(batch[r]) + 1, dtype=np.int64)
                offsets[1:] = np.cumsum([c.size for c in batch[r]])
                d = hc.hits_to_device(hits)
                start.wait()
                for rep in range(3):
                    labels, feats, k = hc.cluster_batch(d, offsets, 128, disorder_hint=512, stream=s2)
                    s2.synchronize()
                    out[("batch", r, rep)] = (labels.cpu().numpy(), feats.cpu().numpy(), k.cpu().numpy(), offsets)
        except Exception as e:
            errors.append(e)
            start.abort()

    for r in range(2):
        print("concurrent round %d" % r, flush=True)
        t1 = threading.Thread(target=run_plain, args=(r,))
        t2 = threading.Thread(target=run_batch, args=(r,))
        t1.start(); t2.start(); t1.join(); t2.join()
        start.reset()
        assert not errors, errors
        for rep in range(3):
            gl, gf = out[("plain", r, rep)]
            wl, wf = want_plain[r]
            assert np.array_equal(gl, wl), "plain round %d rep %d: labels differ" % (r, rep)
            assert gf.tobytes() == wf.tobytes(), "plain round %d rep %d: features differ" % (r, rep)
            lab, fb, k, offsets = out[("batch", r, rep)]
            fb = fb.reshape(-1).view(hc.FEATURE_DTYPE)
            for c, (wl, wf) in enumerate(want_batch[r]):
                a, b = offsets[c], offsets[c + 1]
                assert k[c] == wf.size
                assert np.array_equal(lab[a:b], wl), "batch round %d rep %d chunk %d" % (r, rep, c)
                assert fb[a:a + k[c]].tobytes() == wf.tobytes()
