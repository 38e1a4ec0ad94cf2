"""The oracle's chain has the exact law of isotropic RSA.

* The exact enumerator reproduces rationals computed independently when this
  design was drawn up (a cross-check of the enumerator itself).
* Attempt-based RSA with rejection (uniform site, orientation H/V with
  probability 1/2 each, Sec. II.A) run with numpy's generator has the law the
  enumerator gives: the rejection-free chain is the same process.
* The oracle's empirical laws of n_jam and the wrap steps over many seeds
  match the exact law (chi-square).
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from exact_law import law, mean


def test_enumerator_exact_rationals():
    d = law(3, 2, exact=True)
    assert mean(d["n_jam"]) == Fraction(216, 55)
    assert d["n_jam"] == {3: Fraction(4, 55), 4: Fraction(51, 55)}
    assert mean(d["n_wrap_any"]) == Fraction(29, 11)
    d = law(4, 3, exact=True)
    assert mean(d["n_jam"]) == Fraction(12961, 2850)
    assert d["n_wrap_x"][-1] == Fraction(181, 5700)
    d = law(2, 1, exact=True)
    assert d["n_jam"] == {4: 1}
    assert d["n_wrap_any"] == {2: Fraction(2, 3), 3: Fraction(1, 3)}


def test_enumerator_symmetry_and_proposition():
    for L, k in [(4, 2), (4, 3), (5, 4)]:
        d = law(L, k)
        for v in set(d["n_wrap_x"]) | set(d["n_wrap_y"]):
            assert abs(d["n_wrap_x"].get(v, 0) - d["n_wrap_y"].get(v, 0)) < 1e-12
        assert -1 not in d["n_wrap_any"]  # a cluster wraps by jamming
        assert sum(d["n_jam"].values()) == pytest.approx(1.0)


def _chi2_pvalue(samples, probs, min_expected=5.0):
    n = len(samples)
    values, counts = np.unique(np.asarray(samples), return_counts=True)
    observed = dict(zip(values.tolist(), counts.tolist()))
    assert set(observed) <= set(probs), (set(observed) - set(probs))
    keys = sorted(probs)
    obs, exp = [], []
    o_acc = e_acc = 0.0
    for key in keys:
        o_acc += observed.get(key, 0)
        e_acc += probs[key] * n
        if e_acc >= min_expected:
            obs.append(o_acc)
            exp.append(e_acc)
            o_acc = e_acc = 0.0
    if e_acc > 0:
        obs[-1] += o_acc
        exp[-1] += e_acc
    if len(obs) < 2:
        return 1.0
    return stats.chisquare(obs, exp).pvalue


def _attempt_rsa(L, k, rng):
    occ = np.zeros((L, L), dtype=bool)
    n = 0
    # attempt until no placement fits; check jamming by full scan
    while True:
        fits = []
        for o in (0, 1):
            for y in range(L):
                for x in range(L):
                    cells = [((y + i) % L, x) if o else (y, (x + i) % L) for i in range(k)]
                    if not any(occ[c] for c in cells):
                        fits.append(1)
                        break
                if fits:
                    break
            if fits:
                break
        if not fits:
            return n
        o = rng.integers(2)
        y, x = rng.integers(L), rng.integers(L)
        cells = [((y + i) % L, x) if o else (y, (x + i) % L) for i in range(k)]
        if any(occ[c] for c in cells):
            continue
        for c in cells:
            occ[c] = True
        n += 1


def test_attempt_based_rsa_has_the_enumerated_law():
    rng = np.random.default_rng(1810_06800)
    L, k = 4, 3
    d = law(L, k)
    samples = [_attempt_rsa(L, k, rng) for _ in range(3000)]
    assert _chi2_pvalue(samples, d["n_jam"]) > 1e-4


@pytest.mark.parametrize("L,k,n", [(2, 1, 20000), (3, 2, 40000), (4, 2, 40000), (4, 3, 40000),
                                   (5, 3, 30000), (5, 4, 40000)])
def test_oracle_matches_exact_law(orc, L, k, n):
    d = law(L, k)
    res = orc.run_many([(L, k, 77, s) for s in range(n)])
    assert all(r["status"] == 0 for r in res)
    for field in ("n_jam", "n_wrap_x", "n_wrap_y", "n_wrap_any"):
        p = _chi2_pvalue([r[field] for r in res], d[field])
        assert p > 1e-4, (field, p)
    m = np.mean([r["n_jam"] for r in res])
    sd = np.std([r["n_jam"] for r in res]) / np.sqrt(n)
    assert abs(m - mean(d["n_jam"])) < 5 * sd + 1e-12
