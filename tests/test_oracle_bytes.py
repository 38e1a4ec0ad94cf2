"""Pins of the oracle's changed-word count and of the exact wrap reading.

* ``wchg_words`` (and through it ``alg_bytes``) counts, over all deposits, the
  availability words whose value changes.  The literal reference recomputes
  availability from the occupancy after every deposit (Sec. II.B: every
  placement covering a new site stops being viable) and counts the 64-bit
  words holding a changed placement, with no word bookkeeping of its own.
  The lattices span several words per row (L > 64) and ragged tails.
* Every availability bit goes from 1 to 0 exactly once per run (A_0 in all).
* Sec. II.D tests a cycle closed by the new k-mer with |x1-x2| + |y1-y2| > 2k
  on the unwrapped coordinates of the two sites it touches.  For L > 3k+1 this
  fires at exactly the pairs whose exact winding is non-zero, and the first
  step it fires at is the oracle's n_wrap_any.
"""
import pytest

import literal_ref


@pytest.mark.parametrize("L", list(range(1, 13)))
def test_changed_words_every_small_shape(orc, L):
    for k in range(1, L + 1):
        for seed, sample in ((0, 0), (5, 3)):
            want = literal_ref.word_changes(L, k, seed, sample)
            got = orc.run(L, k, seed, sample)
            assert got["n_jam"] == want["n_jam"]
            assert got["wchg_words"] == want["wchg_words"], (L, k, seed, sample)
            assert want["bits_cleared"] == 2 * L * L


@pytest.mark.parametrize("L,k", [(65, 1), (65, 7), (70, 10), (100, 3), (127, 16), (130, 9),
                                 (129, 64), (150, 40), (192, 12), (200, 100)])
def test_changed_words_multiword_rows(orc, L, k):
    for sample in range(2):
        want = literal_ref.word_changes(L, k, 77, sample)
        got = orc.run(L, k, 77, sample)
        assert got["n_jam"] == want["n_jam"]
        assert got["wchg_words"] == want["wchg_words"], (L, k, sample)
        wd = (L + 63) // 64
        base = 4 * L * L + 16 * L * wd
        per = 4 * k + 4 * (2 * k + 2) + 8 * wd + 16
        assert got["alg_bytes"] == base + got["n_jam"] * per + 16 * want["wchg_words"]


def test_changed_words_h_only_rings(orc):
    for L, k in ((66, 5), (100, 2)):
        want = literal_ref.word_changes(L, k, 3, 1, h_only=True)
        got = orc.run(L, k, 3, 1, flags=1)
        assert got["wchg_words"] == want["wchg_words"]
        assert want["bits_cleared"] == L * L


@pytest.mark.parametrize("L,k", [(5, 1), (8, 2), (11, 3), (12, 2), (14, 4), (17, 5), (20, 6)])
def test_paper_2k_test_equals_exact_winding(orc, L, k):
    assert L > 3 * k + 1
    for sample in range(4):
        got = literal_ref.paper_wrap_test(L, k, 1810, sample)
        want = orc.run(L, k, 1810, sample)
        assert got["pairs"] > 0
        assert got["disagree"] == 0, (L, k, sample)
        assert got["first_2k"] == want["n_wrap_any"], (L, k, sample)


def test_paper_2k_test_differs_on_small_tori():
    # at L <= 3k + 1 a short cycle that winds can stay within 2k: the exact
    # winding is needed there (so the library never relies on the 2k test)
    bad = 0
    for L, k in ((4, 2), (5, 2), (7, 2), (7, 3)):
        for sample in range(6):
            bad += literal_ref.paper_wrap_test(L, k, 1810, sample)["disagree"]
    assert bad > 0
