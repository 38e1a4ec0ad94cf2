"""Pins of the oracle's statistics beyond the two thresholds: the contact
census at jamming (Eq. 12: n_x, n_y, n_xy) and the cluster-size histogram
right after a chosen deposit (Eq. 11: n_s at the percolation threshold).

The literal reference gives both by brute force from its own occupancy grid
(neighbour pairs site by site; clusters by breadth-first search), on every
small torus; identities that hold at any size pin the rest.
"""
import pytest

import literal_ref


def brute_contacts(L, k, seed, sample, h_only=False):
    lit = literal_ref.run(L, k, seed, sample, h_only=h_only)
    return literal_ref.contacts(lit["owner"], lit["orient"])


@pytest.mark.parametrize("L", list(range(1, 10)))
def test_contacts_match_brute_force(orc, L):
    for k in range(1, L + 1):
        for seed, sample in ((0, 0), (5, 3)):
            assert orc.contacts_at_jamming(L, k, seed, sample) == brute_contacts(L, k, seed, sample), (L, k)


def test_contacts_h_only_and_identities(orc):
    # only horizontal needles: neither vertical nor perpendicular contacts
    for L, k in ((8, 3), (9, 2), (12, 4)):
        for sample in range(3):
            got = orc.contacts_at_jamming(L, k, 11, sample, flags=1)
            assert got == brute_contacts(L, k, 11, sample, h_only=True)
            assert got[1] == 0 and got[2] == 0 and got[0] > 0
    # k = 1 fills every site with its own k-mer: each of the 2L^2 neighbour
    # pairs (right and down of every site) is a contact
    for L in (2, 3, 7, 16, 40):
        assert sum(orc.contacts_at_jamming(L, 1, 3, 0)) == 2 * L * L
    # k = L: L parallel needles fill the torus, every pair across them is a
    # contact between needles of one orientation
    for L in (4, 7, 10):
        nx, ny, nxy = orc.contacts_at_jamming(L, L, 9, 1)
        assert nxy == 0 and nx + ny == L * L and (nx == 0 or ny == 0)


def test_contacts_larger_brute_force(orc):
    for L, k, sample in ((16, 3, 0), (20, 4, 1), (24, 6, 2)):
        assert orc.contacts_at_jamming(L, k, 77, sample) == brute_contacts(L, k, 77, sample)


@pytest.mark.parametrize("L,k", [(6, 2), (8, 3), (9, 2), (10, 4), (12, 3), (12, 1)])
def test_snapshot_histogram_matches_bfs(orc, L, k):
    for sample in range(3):
        lit = literal_ref.run(L, k, 21, sample)
        for step in sorted({lit["n_wrap_any"], max(1, lit["n_jam"] // 2), lit["n_jam"]}):
            want = literal_ref.run(L, k, 21, sample, snap_step=step)["snap_hist"]
            got = orc.run(L, k, 21, sample, snap_step=step, snap_cap=L * L + 1)["snap_hist"]
            assert {s: n for s, n in enumerate(got) if n} == want, (L, k, sample, step)
            # every occupied site is in exactly one cluster
            assert sum(s * n for s, n in enumerate(got)) == step * k
