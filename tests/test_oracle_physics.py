"""Special cases, the paper's invariants and its printed statistics.

* k = 1: every site ends occupied (p_j = 1, Table I row n = 0).
* k = L: each k-mer fills a whole row or column; n_jam = L, the first k-mer
  wraps itself, the other direction closes with the last.
* Appendix A: every cluster of a jammed torus wraps; p_c <= p_j.
* Table I (single runs at L = 100k): the oracle's mean p_c, p_j at the same
  L/k agree within the spread of a single run.
* Appendix A quotes R* = 0.521058290 for the probability of a horizontal wrap
  at p_c: for k = 1 the fraction of samples wrapped in x after
  round(p_c L^2) deposits is close to it.
"""
import math
import os
import random

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1_pc_pj.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, pc, pj = line.split()
                rows[int(n)] = (float(pc), float(pj))
    return rows


@pytest.mark.parametrize("L", [1, 2, 3, 7, 16, 33])
def test_k1_fills_every_site(orc, L):
    for s in range(3):
        r = orc.run(L, 1, 11, s)
        assert r["status"] == 0
        assert r["n_jam"] == L * L


@pytest.mark.parametrize("L", [1, 2, 3, 5, 16, 64])
def test_k_equals_L(orc, L):
    for s in range(4):
        r = orc.run(L, L, 3, s)
        assert r["status"] == 0
        assert r["n_jam"] == L
        assert r["n_wrap_any"] == 1
        if L > 1:
            assert sorted((r["n_wrap_x"], r["n_wrap_y"])) == [1, L]


def test_invariants_random_shapes(orc):
    rng = random.Random(42)
    descs = []
    for _ in range(300):
        L = rng.randint(1, 40)
        k = rng.randint(1, L)
        descs.append((L, k, rng.getrandbits(64), rng.getrandbits(32)))
    res = orc.run_many(descs)
    for d, r in zip(descs, res):
        L, k = d[0], d[1]
        assert r["status"] == 0, (d, r["status"])
        assert r["n_jam"] * k <= L * L
        assert 1 <= r["n_wrap_any"] <= r["n_jam"]
        assert r["n_clusters_jam"] >= 1
        assert r["n_nonwrapping_jam"] == 0


def test_algorithmic_bytes_bounds(orc):
    # each availability bit is cleared exactly once per run, so the number of
    # changed words lies between the number of nonzero words and the bits
    for L, k in [(64, 8), (100, 3), (257, 16)]:
        r = orc.run(L, k, 1, 0)
        wd = (L + 63) // 64
        assert 2 * L * wd <= r["wchg_words"] <= 2 * L * L
        base = 4 * L * L + 16 * L * wd
        per = 4 * k + 4 * (2 * k + 2) + 8 * wd + 16
        assert r["alg_bytes"] == base + r["n_jam"] * per + 16 * r["wchg_words"]


@pytest.mark.parametrize("n,samples", [(0, 48), (1, 24), (2, 16), (3, 12), (4, 8)])
def test_table1_rows_at_paper_size(orc, n, samples):
    k = 2 ** n
    L = 100 * k
    pc_paper, pj_paper = table1()[n]
    res = orc.run_many([(L, k, 1810, s) for s in range(samples)])
    assert all(r["status"] == 0 for r in res)
    pc = np.array([r["n_wrap_any"] * k / L**2 for r in res])
    pj = np.array([r["n_jam"] * k / L**2 for r in res])
    # the paper's entry is one run at the same L: compare within the spread
    # of a single run (plus the spread of our mean)
    grow = math.sqrt(1 + 1 / samples)
    assert abs(pc.mean() - pc_paper) < 4.5 * pc.std(ddof=1) * grow + 1e-3
    assert abs(pj.mean() - pj_paper) < 4.5 * pj.std(ddof=1) * grow + 1e-3
    if n == 0:
        assert np.all(pj == 1.0)


def test_horizontal_wrap_probability_at_pc(orc):
    with open(os.path.join(GOLDEN, "wrap_probability.txt")) as f:
        rstar = float([ln for ln in f if ln.startswith("R_star")][0].split()[1])
    pc = table1()[0][0]
    L, n = 96, 3000
    res = orc.run_many([(L, 1, 52, s) for s in range(n)])
    steps = round(pc * L * L)
    frac = np.mean([0 < r["n_wrap_x"] <= steps for r in res])
    assert abs(frac - rstar) < 4 * math.sqrt(rstar * (1 - rstar) / n) + 0.01
    # and either-direction wrapping happens no later than x or y alone
    assert all(r["n_wrap_any"] == min(v for v in (r["n_wrap_x"], r["n_wrap_y"]) if v > 0)
               for r in res)
