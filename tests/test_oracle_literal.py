"""Oracle vs the literal reference on every tiny torus.

The literal reference recomputes the available placements from the occupancy
and the wrap state by a breadth-first winding search after every deposit, so
any slip in the oracle's bookkeeping (row counts, strip/block clears, seams,
contact vectors, relabelling shifts) changes a placement, a wrap step or the
hash on some (L, k, seed, sample).
"""
import pytest

import literal_ref

FIELDS = ("n_jam", "n_wrap_x", "n_wrap_y", "n_wrap_any", "occ_hash", "seq_hash", "seq",
          "n_clusters_jam", "n_nonwrapping_jam")


def _compare(orc, L, k, seed, sample, h_only=False):
    want = literal_ref.run(L, k, seed, sample, h_only=h_only)
    got = orc.run(L, k, seed, sample, flags=1 if h_only else 0, want_seq=True)
    assert got["status"] == 0
    for f in FIELDS:
        assert got[f] == want[f], (L, k, seed, sample, f)


@pytest.mark.parametrize("L", list(range(1, 13)))
def test_every_k_small_lattices(orc, L):
    seeds = [(0, 0), (1, 7), (0xDEADBEEFCAFEF00D, 12345)]
    for k in range(1, L + 1):
        for seed, sample in seeds:
            _compare(orc, L, k, seed, sample)


@pytest.mark.parametrize("L,k", [(8, 3), (9, 2), (12, 4), (5, 5)])
def test_h_only_rings_literal(orc, L, k):
    for sample in range(4):
        _compare(orc, L, k, 99, sample, h_only=True)


def test_many_seeds_medium(orc):
    for L, k in [(16, 2), (16, 5), (20, 3), (24, 8)]:
        for sample in range(3):
            _compare(orc, L, k, 2024, sample)
