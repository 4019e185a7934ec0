"""The pins are not vacuous: each plausible mistake, planted in a copy of the
oracle's source and compiled on the CPU, must be caught by at least one pin."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()

# (name, original text, replacement) -- each a single plausible slip
MUTANTS = [
    ("no_own_pixel",
     "if (qx < 0 || qx >= (int64_t)width) continue;",
     "if (qx < 0 || qx >= (int64_t)width || (qx == hx && qy == hy)) continue;"),
    ("strict_dt",
     "hits[list[k]].toa <= hi",
     "hits[list[k]].toa < hi"),
    ("missing_right_column",
     "for (int64_t qx = hx - 1; qx <= hx + 1; qx++)",
     "for (int64_t qx = hx - 1; qx <= hx; qx++)"),
    ("four_neighbourhood",
     "if (qx < 0 || qx >= (int64_t)width) continue;",
     "if (qx < 0 || qx >= (int64_t)width || (qx != hx && qy != hy)) continue;"),
    ("row_major_wraparound",
     "if (qx < 0 || qx >= (int64_t)width) continue;",
     "if (qy * (int64_t)width + qx < 0 || qy * (int64_t)width + qx >= npix) continue;"),
    ("label_is_largest_index",
     "for (int64_t seed = 0; seed < n; seed++) {",
     "for (int64_t seed = n - 1; seed >= 0; seed--) {"),
    ("unsaturated_window_low",
     "uint64_t lo = sat_sub(hits[h].toa, dt)",
     "uint64_t lo = hits[h].toa - dt"),
    ("unsaturated_window_high",
     "hi = sat_add(hits[h].toa, dt);",
     "hi = hits[h].toa + dt;"),
    ("centroid_swapped_axes",
     "f->cx = (double)sxt[c] / (double)st[c];",
     "f->cx = (double)syt[c] / (double)st[c];"),
    ("centroid_unweighted",
     "f->cy = (double)syt[c] / (double)st[c];",
     "f->cy = (double)sy[c] / (double)size[c];"),
    ("toa_max_last_seen",
     "if (hits[i].toa > tmax[c]) tmax[c] = hits[i].toa;",
     "tmax[c] = hits[i].toa;"),
    ("sum_tot_dropped_term",
     "st[c] += t;",
     "st[c] += (t > 1 ? t - 1 : t);"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new):
    assert SRC.count(old) >= 1, "mutation anchor missing: %s" % name
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "mutant.c")
        so = os.path.join(d, "libmutant.so")
        open(src, "w").write(SRC.replace(old, new, 1))
        oracle.build(src, so)
        # run the pins in a child process: a mutant may also crash outright
        here = os.path.dirname(os.path.abspath(__file__))
        code = ("import sys; sys.path[:0] = [%r, %r]\n"
                "import oracle, pins\n"
                "lib = oracle.load(%r)\n"
                "bad = []\n"
                "for p in pins.PINS:\n"
                "    try:\n"
                "        p(lib)\n"
                "    except Exception as e:\n"
                "        bad.append(p.__name__)\n"
                "print('caught by', bad)\n"
                "sys.exit(1 if bad else 0)\n") % (here, os.path.dirname(here), so)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, "mutant %s passed every pin: %s" % (name, r.stdout)
