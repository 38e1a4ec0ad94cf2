"""Exact law of one RSA run on a tiny torus, by enumeration of occupancy states.

Test tool, independent of the oracle.  The chain is the one the method
defines: from an occupancy state, the next k-mer is uniform over the available
(o, y, x) placements (isotropic RSA conditioned on success, Sec. II.A-II.B);
the state is jammed when none is left.  Clusters, and whether one wraps, are
functions of the occupancy alone (4-neighbour adjacency of occupied sites), so
P(n_x <= t) = P(the state after min(t, n_jam) deposits wraps in x), because a
wrap, once present, stays.

Probabilities are exact fractions when ``exact=True`` (slow), floats otherwise.
"""
from __future__ import annotations

from collections import defaultdict
from fractions import Fraction
from functools import lru_cache

import numpy as np

from literal_ref import clusters_and_windings


def _placements(L: int, k: int, h_only: bool):
    out = []
    for o in (0, 1):
        if o == 1 and h_only:
            continue
        for y in range(L):
            for x in range(L):
                m = 0
                for i in range(k):
                    sy, sx = ((y + i) % L, x) if o else (y, (x + i) % L)
                    m |= 1 << (sy * L + sx)
                out.append(m)
    return out


def law(L: int, k: int, h_only: bool = False, exact: bool = False) -> dict:
    """Distributions of n_jam, n_wrap_x, n_wrap_y, n_wrap_any as dicts
    value -> probability (value -1 = never)."""
    places = _placements(L, k, h_only)
    one = Fraction(1) if exact else 1.0
    zero = 0 * one

    @lru_cache(maxsize=None)
    def info(state: int):
        avail = tuple(m for m in places if m & state == 0)
        occ = np.array([(state >> s) & 1 for s in range(L * L)], dtype=bool).reshape(L, L)
        _, cl = clusters_and_windings(occ)
        return avail, any(c[1] for c in cl), any(c[2] for c in cl)

    dist = {0: one}
    cdf = {"n_jam": [], "n_wrap_x": [], "n_wrap_y": [], "n_wrap_any": []}
    while True:
        acc = {name: zero for name in cdf}
        live = False
        for st, p in dist.items():
            avail, wx, wy = info(st)
            if not avail:
                acc["n_jam"] += p
            else:
                live = True
            if wx:
                acc["n_wrap_x"] += p
            if wy:
                acc["n_wrap_y"] += p
            if wx or wy:
                acc["n_wrap_any"] += p
        for name in cdf:
            cdf[name].append(acc[name])
        if not live:
            break
        nxt = defaultdict(lambda: zero)
        for st, p in dist.items():
            avail = info(st)[0]
            if not avail:
                nxt[st] += p
                continue
            share = p / len(avail)
            for m in avail:
                nxt[st | m] += share
        dist = dict(nxt)

    out = {}
    for name, c in cdf.items():
        d = {}
        prev = zero
        for step, v in enumerate(c):
            if v != prev:
                d[step] = v - prev
            prev = v
        never = one - c[-1]
        if (exact and never != 0) or (not exact and never > 1e-12):
            d[-1] = never
        out[name] = d
    return out


def mean(d: dict):
    return sum(key * val for key, val in d.items())
