"""The served form at its stated size, in the configuration bench.py times:
8 detector streams of 256x256 at 37.5 Mhit/s each (Poisson chunk arrivals,
aggregate 300 Mhit/s, chunks log-uniform in [4k, 1M] hits) for 10 s under a
16 GiB budget.  Every stream replays a 4M-hit pool with a ToA offset per pass,
so the oracle on the pool gives the expected labels of every pass (offset by
the hits of the earlier passes); every label of every pass that was served is
compared, element by element."""
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_served_10s_labels_match_oracle():
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import paper_2412_11809_amd as hc
    sys.path.insert(0, ROOT)
    import bench
    import hitgen
    assert torch.cuda.is_available()
    hc.load_library()
    pool = 4_000_000
    pools, _, _ = bench._served_pools(8, pool, hitgen.BASE_SEED + 5)
    with ThreadPoolExecutor(8) as ex:
        want = list(ex.map(lambda h: oracle.cluster(h, 256, 256, 128, features=False)[0], pools))
    seen = {"hits": 0, "passes": 0}
    prefix_cache = {}

    def check_pass(s, p, n_hits, labels):
        if n_hits == pool:
            w = want[s]
        else:  # the run ended inside this pass: the oracle of the submitted prefix
            key = (s, n_hits)
            if key not in prefix_cache:
                prefix_cache[key] = oracle.cluster(pools[s][:n_hits], 256, 256, 128, features=False)[0]
            w = prefix_cache[key]
        got = labels[:n_hits].astype(np.int64) - p * pool
        bad = np.nonzero(got != w)[0]
        assert bad.size == 0, "stream %d pass %d: %d labels differ (first %s)" % (s, p, bad.size, bad[:5])
        seen["hits"] += n_hits
        seen["passes"] += 1

    dev = torch.device("cuda:0")
    out = bench.bench_served(hc, torch, dev, 10.0, check_pass=check_pass, rate_only=True)
    print(out, seen, flush=True)
    assert out["rejected"] == 0
    assert seen["hits"] == out["hits_served"], "every served hit was checked"
    assert out["hits_served"] >= 2_000_000_000  # about 10 s at 300 Mhit/s
    assert seen["passes"] >= 8 * (out["hits_served"] // (8 * pool))
