"""H_ONLY mode: every row is an independent ring of length L (1D RSA).

Pins: the mean number of empty sites of 1D RSA on an open segment obeys
E_n = n (n < k), E_n = 2/(n-k+1) * sum_{j<=n-k} E_j; a ring of length L
leaves E_open(L-k) empty sites after its first k-mer.  For k = 2 the jammed
coverage tends to Flory's 1 - e^-2; for general k to the classical integral
theta_k = k * int_0^inf exp(-u - 2 sum_{j<k} (1 - e^{-ju})/j) du.
"""
import math

import numpy as np
import pytest
from scipy import integrate


def empty_open(n_max, k):
    E = [0.0] * (n_max + 1)
    prefix = [0.0] * (n_max + 2)
    for n in range(n_max + 1):
        if n < k:
            E[n] = float(n)
        else:
            E[n] = 2.0 / (n - k + 1) * prefix[n - k + 1]
        prefix[n + 1] = prefix[n] + E[n]
    return E


def ring_coverage(L, k):
    return 1.0 - empty_open(L, k)[L - k] / L


def theta(k):
    f = lambda u: math.exp(-u - 2.0 * sum((1.0 - math.exp(-j * u)) / j for j in range(1, k)))
    val, _ = integrate.quad(f, 0, math.inf, limit=200)
    return k * val


def test_recursion_reaches_flory_limit():
    assert ring_coverage(4096, 2) == pytest.approx(1 - math.exp(-2), abs=1e-12)
    assert theta(2) == pytest.approx(1 - math.exp(-2), abs=1e-10)


@pytest.mark.parametrize("k,ref", [(3, 0.823653), (4, 0.803893), (8, 0.775185)])
def test_recursion_matches_integral(k, ref):
    assert theta(k) == pytest.approx(ref, abs=2e-6)
    # finite rings approach the limit like 1/L
    assert ring_coverage(20000, k) == pytest.approx(theta(k), abs=5.0 * k / 20000)


@pytest.mark.parametrize("L,k", [(64, 2), (64, 3), (48, 8), (32, 32), (33, 16)])
def test_oracle_h_only_mean_coverage(orc, L, k):
    n = 400
    res = orc.run_many([(L, k, 5, s, orc.FLAG_H_ONLY) for s in range(n)])
    assert all(r["status"] == 0 for r in res)
    nj = np.array([r["n_jam"] for r in res], dtype=float)
    expect = L * L * ring_coverage(L, k) / k  # E[n_jam], L independent rings
    assert abs(nj.mean() - expect) < 5 * nj.std() / math.sqrt(n) + 1e-9
    # every row is its own ring: no vertical contact can ever wrap in x
    # unless a ring closes on itself, which needs k-mers to fill it
    assert all(r["n_wrap_any"] >= 1 for r in res)
