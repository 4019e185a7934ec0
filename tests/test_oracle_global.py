"""Pins of the Section 2 (iii)(b) oracle (oracle_global.c): exhaustive brute
force over every subset of tiny inputs (the maximal sets that are spatially
connected and leave no ToA gap above dt), the hand-derived fixture, what the
definition fixes in closed form, its relation to the (iii)(a) clusters, and
planted mistakes that the pins must catch."""
import itertools
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import hitgen
import oracle
from pins import load_golden

HERE = os.path.dirname(os.path.abspath(__file__))
U64MAX = (1 << 64) - 1


def valid(hits, members, dt):
    """(ii) spatial connectivity inside the set and (iii)(b) no ToA gap > dt."""
    m = list(members)
    toa = sorted(int(hits["toa"][i]) for i in m)
    if any(b - a > dt for a, b in zip(toa, toa[1:])):
        return False
    seen, todo = {m[0]}, [m[0]]
    while todo:
        h = todo.pop()
        for j in m:
            if j not in seen and abs(int(hits["x"][h]) - int(hits["x"][j])) <= 1 and \
                    abs(int(hits["y"][h]) - int(hits["y"][j])) <= 1:
                seen.add(j)
                todo.append(j)
    return len(seen) == len(m)


def brute_global(hits, dt):
    n = hits.size
    ok = [frozenset(c) for r in range(1, n + 1) for c in itertools.combinations(range(n), r) if valid(hits, c, dt)]
    maximal = [c for c in ok if not any(c < d for d in ok)]
    labels = np.full(n, -1, dtype=np.int64)
    for c in maximal:
        assert (labels[list(c)] == -1).all(), "maximal sets overlap"
        labels[list(c)] = min(c)
    assert (labels >= 0).all()
    return labels


def random_tiny(rng):
    n = int(rng.integers(1, 10))
    h = np.zeros(n, dtype=hitgen.HIT_DTYPE)
    h["x"] = rng.integers(0, int(rng.integers(1, 5)), n)
    h["y"] = rng.integers(0, int(rng.integers(1, 5)), n)
    h["toa"] = rng.integers(0, int(rng.integers(1, 60)), n)
    return h, int(rng.integers(0, 25))


def pin_bruteforce(lib, cases=400, seed=3):
    rng = np.random.default_rng(seed)
    for _ in range(cases):
        h, dt = random_tiny(rng)
        got, _ = oracle.cluster_global(h, 8, 8, dt, features=False, lib=lib)
        assert np.array_equal(got, brute_global(h, dt)), (h, dt)


def pin_golden(lib):
    w, h_, dt, hits, want, _ = load_golden(os.path.join(HERE, "golden", "variant_b", "global_time.txt"))
    got, _ = oracle.cluster_global(hits, w, h_, dt, features=False, lib=lib)
    assert got.tolist() == want.tolist()


def pin_closed_forms(lib):
    rng = np.random.default_rng(5)
    # one pixel: the clusters are the runs between ToA gaps above dt, as under (iii)(a)
    h = np.zeros(300, dtype=hitgen.HIT_DTYPE)
    h["toa"] = np.sort(rng.integers(0, 3000, 300))
    rng.shuffle(h)
    got, _ = oracle.cluster_global(h, 4, 4, 7, features=False, lib=lib)
    want, _ = oracle.cluster(h, 4, 4, 7, features=False)
    assert np.array_equal(got, want)
    # dt = infinity: spatial components of the occupied pixels
    h = hitgen.uniform_hits(500, 6, width=40, height=40, toa_hi=10 ** 6)
    got, _ = oracle.cluster_global(h, 40, 40, U64MAX, features=False, lib=lib)
    want, _ = oracle.cluster(h, 40, 40, U64MAX, features=False)
    assert np.array_equal(got, want)
    # dt = 0 on distinct ToAs: nothing joins
    h = np.zeros(50, dtype=hitgen.HIT_DTYPE)
    h["toa"] = rng.permutation(50) * 3
    got, k = oracle.cluster_global(h, 2, 2, 0, features=False, lib=lib)
    assert k == 50 and np.array_equal(got, np.arange(50))


def pin_refines(lib):
    """Every (iii)(a) cluster is spatially connected and gap-free, so it lies
    inside one (iii)(b) cluster; with dt large against the clusters' spans the
    two agree."""
    hits, p = hitgen.mixed_10m(n=40_000, seed=12)
    a, _ = oracle.cluster(hits, 256, 256, p["dt"], features=False)
    b, _ = oracle.cluster_global(hits, 256, 256, p["dt"], features=False, lib=lib)
    for lab in np.unique(a):
        assert np.unique(b[a == lab]).size == 1
    assert np.unique(b).size <= np.unique(a).size


def pin_metamorphic(lib):
    rng = np.random.default_rng(8)
    h = hitgen.uniform_hits(3000, 9, width=30, height=30, toa_hi=4000)
    base, _ = oracle.cluster_global(h, 30, 30, 9, features=False, lib=lib)

    def same_partition(l1, l2):
        _, i1 = np.unique(l1, return_inverse=True)
        _, i2 = np.unique(l2, return_inverse=True)
        pairs = set(zip(i1.tolist(), i2.tolist()))
        return len(pairs) == np.unique(i1).size == np.unique(i2).size

    perm = rng.permutation(h.size)
    l2, _ = oracle.cluster_global(h[perm], 30, 30, 9, features=False, lib=lib)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    assert same_partition(base, l2[inv])
    h2 = h.copy()
    h2["toa"] += np.uint64(123456789)
    h2["x"] = 29 - h2["x"]
    l3, _ = oracle.cluster_global(h2, 30, 30, 9, features=False, lib=lib)
    assert np.array_equal(base, l3)


PINS = [pin_bruteforce, pin_golden, pin_closed_forms, pin_refines, pin_metamorphic]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(oracle.load())


def test_features_are_the_feature_definition():
    hits, p = hitgen.mixed_10m(n=30_000, seed=13)
    labels, feats = oracle.cluster_global(hits, 256, 256, p["dt"])
    # the numpy feature step agrees with oracle.c's on (iii)(a) labels ...
    la, fa = oracle.cluster(hits, 256, 256, p["dt"])
    assert oracle.features_from_labels(hits, la).tobytes() == fa.tobytes()
    # ... and sizes and sums add up on the (iii)(b) clusters
    assert feats["size"].sum() == hits.size
    assert feats["sum_tot"].sum() == hits["tot"].astype(np.uint64).sum()


SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle_global.c")).read()
MUTANTS = [
    ("strict_gap", "recs[k].key - recs[k - 1].key > dt", "recs[k].key - recs[k - 1].key >= dt"),
    ("no_own_pixel", "if (qx < 0 || qx >= (int64_t)width) continue;",
     "if (qx < 0 || qx >= (int64_t)width || (qx == hx && qy == hy)) continue;"),
    ("one_round_only", "if (count == n_parts) break;", "break;"),
    ("four_neighbourhood", "if (qx < 0 || qx >= (int64_t)width) continue;",
     "if (qx < 0 || qx >= (int64_t)width || (qx != hx && qy != hy)) continue;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    assert SRC.count(old) == 1, "mutation anchor missing: %s" % name
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "mutant_global.c")
        so = os.path.join(d, "libmutant.so")
        open(src, "w").write(SRC.replace(old, new, 1))
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", so,
                               os.path.join(os.path.dirname(oracle.__file__), "oracle.c"), src])
        code = ("import sys; sys.path[:0] = [%r, %r]\n"
                "import oracle, test_oracle_global as t\n"
                "lib = oracle.load(%r)\n"
                "bad = []\n"
                "for p in t.PINS:\n"
                "    try:\n"
                "        p(lib)\n"
                "    except Exception:\n"
                "        bad.append(p.__name__)\n"
                "print('caught by', bad)\n"
                "sys.exit(1 if bad else 0)\n") % (HERE, os.path.dirname(HERE), so)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, "mutant %s passed every pin: %s" % (name, r.stdout)
