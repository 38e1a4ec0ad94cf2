"""Pins of the oracle's building blocks: Philox4x32-10, the rank draw, mix64.

Philox is pinned against rocRAND, an independent implementation of the
published generator (Salmon et al., SC'11), compiled here for the host only.
"""
import os
import random
import shutil
import subprocess

import pytest

import literal_ref

HERE = os.path.dirname(os.path.abspath(__file__))
MASK64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND pin")
    exe = str(tmp_path_factory.mktemp("philox") / "philox_rocrand")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "philox_rocrand.cpp")])

    def run(cases):
        text = "".join(f"{s} {c[0]} {c[1]} {c[2]} {c[3]}\n" for s, c in cases)
        out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout
        return [tuple(int(v) for v in line.split()) for line in out.splitlines()]

    return run


def _cases(n=400):
    rng = random.Random(20181016)
    cases = [(0, (0, 0, 0, 0)), (MASK64, (0xFFFFFFFF, (1 << 30) - 1, 0xFFFFFFFF, 0xFFFFFFFF))]
    # the layout the method uses: counter (t, sample, 0, 0), key = seed
    for _ in range(n):
        cases.append((rng.getrandbits(64), (rng.getrandbits(32), rng.getrandbits(30), 0, 0)))
    for _ in range(n // 4):
        cases.append((rng.getrandbits(64), (rng.getrandbits(32), rng.getrandbits(30),
                                            rng.getrandbits(32), rng.getrandbits(32))))
    for seed in range(4):
        for t in range(8):
            cases.append((seed, (t, 3, 0, 0)))
    return cases


def test_oracle_philox_matches_rocrand(orc, rocrand_philox):
    cases = _cases()
    want = rocrand_philox(cases)
    for (seed, ctr), w in zip(cases, want):
        got = orc.philox(ctr, (seed & 0xFFFFFFFF, seed >> 32))
        assert got == w, (seed, ctr)


def test_literal_reference_philox_matches_rocrand(rocrand_philox):
    cases = _cases(100)
    want = rocrand_philox(cases)
    for (seed, ctr), w in zip(cases, want):
        assert literal_ref.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32)) == w


def test_rank_is_floor_u_times_a_over_2_64(orc):
    rng = random.Random(7)
    us = [0, 1, MASK64, MASK64 - 1, 1 << 63, (1 << 63) - 1, 1 << 32, (1 << 32) - 1]
    us += [rng.getrandbits(64) for _ in range(2000)]
    As = [1, 2, 3, 63, 64, 65, (1 << 31) - 1, 1 << 31, 0xFFFFFFFF]
    As += [rng.randrange(1, 1 << 32) for _ in range(50)]
    for u in us[:200]:
        for a in As:
            r = orc.rank(u, a)
            assert r == (u * a) >> 64
            assert 0 <= r < a
    for u in us:
        a = rng.randrange(1, 1 << 32)
        assert orc.rank(u, a) == (u * a) >> 64


def test_rank_is_uniform_enough():
    # floor(u*A/2^64) hits each of the A values 2^64/A times up to one: the
    # largest relative bias is below A/2^64.
    for a in (3, 1000, (1 << 31) + 7):
        lo, hi = (1 << 64) // a, -(-(1 << 64) // a)
        assert hi - lo <= 1


def test_mix64_splitmix64_sequence(orc):
    # SplitMix64 seeded with 0 (Steele, Lea, Flood 2014): the first output is
    # the finalizer applied to the golden-gamma increment.
    gamma = 0x9E3779B97F4A7C15
    assert orc.mix64(gamma) == 0xE220A8397B1DCDAF
    state = 0
    outs = []
    for _ in range(3):
        state = (state + gamma) & MASK64
        outs.append(orc.mix64(state))
    assert outs[0] == 0xE220A8397B1DCDAF
    assert len(set(outs)) == 3


def _unxorshift(z, s):
    x = z
    for _ in range(64 // s + 1):
        x = z ^ (x >> s)
    return x & MASK64


def test_mix64_is_a_bijection(orc):
    # invert each step: multiply by the inverse odd constant, undo the xorshift
    inv1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    inv2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    rng = random.Random(3)
    for z in [0, 1, MASK64] + [rng.getrandbits(64) for _ in range(500)]:
        h = orc.mix64(z)
        x = _unxorshift(h, 31)
        x = (x * inv2) & MASK64
        x = _unxorshift(x, 27)
        x = (x * inv1) & MASK64
        x = _unxorshift(x, 30)
        assert x == z
        assert literal_ref.mix64(z) == h
