"""GPU: the request server (continuous batching with time-sliced launches),
through the C ABI, against the oracle and against rsa_run_batch.

A sample that yields saves its row counts and chain position and resumes
exactly there, so every result must be bit-exact whatever the quantum, the
arena size or the other requests beside it.
"""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("n_jam", "n_wrap_x", "n_wrap_y", "n_wrap_any", "occ_hash", "seq_hash",
          "alg_bytes", "wchg_words", "n_clusters_jam", "n_nonwrapping_jam", "status",
          "n_contacts_x", "n_contacts_y", "n_contacts_xy")
CONTACTS = ("n_contacts_x", "n_contacts_y", "n_contacts_xy")
CENSUS = ("n_clusters_jam", "n_nonwrapping_jam")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_1810_06800_amd import rsa

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = rsa.Context(0)
    yield c
    c.close()


def same(got, want):
    """Field by field, census included (both sides from the library)."""
    bad = [(i, f, g[f], w[f]) for i, (g, w) in enumerate(zip(got, want)) for f in FIELDS if g[f] != w[f]]
    assert not bad, f"{len(bad)} mismatches, first: {bad[:5]}"


def same_as_oracle(descs, got, want):
    """Against the oracle, which always takes the census: the library reports
    it only for RSA_FLAG_TRACK_CLUSTERS samples (-1 otherwise)."""
    bad = []
    for i, (d, g, w) in enumerate(zip(descs, got, want)):
        assert w["status"] == 0
        for f in FIELDS:
            if f in CONTACTS:
                continue
            expect = w[f] if (f not in CENSUS or d[4] & 2) else -1
            if g[f] != expect:
                bad.append((d, f, g[f], expect))
    assert not bad, f"{len(bad)} mismatches, first: {bad[:5]}"


# one request per schedule family: 1, 2, 3 and 7 selecting waves, wide rows,
# the sparse clear, H-only rings and the cluster census
MIX = [
    [(64, 8, 1, s, 0) for s in range(6)],
    [(200, 20, 3, 1, 2), (300, 7, 8, 2, 0)],
    [(512, 128, 4, s, 0) for s in range(2)],
    [(700, 250, 5, 0, 2)],
    [(1100, 512, 6, 0, 0)],
    [(4160, 64, 7, 0, 0)],
    [(96, 4, 9, s, 1) for s in range(3)],
    [(1024, 64, 10, s, 0) for s in range(3)],
    [(150, 10, 12, s, 4) for s in range(2)],
]


def test_time_sliced_runs_are_exact(ctx, orc):
    """A 20 us quantum makes every sample yield and resume many times."""
    from paper_1810_06800_amd import rsa

    _log("server: 8 requests, quantum 20 us")
    with rsa.Server(ctx, arena_bytes=1 << 30, quantum_us=20) as srv:
        got = srv.run(MIX)
        # a finished sample's slab is freed once the last launch listing it
        # (at most one launch behind) has been retired
        for _ in range(4):
            srv.step(wait=True)
        st = srv.stats()
    _log(f"server stats: {st}")
    flat = [d for r in MIX for d in r]
    want = orc.run_many(flat, threads=min(16, os.cpu_count() or 1))
    same_as_oracle(flat, [g for r in got for g in r], want)
    for d, g in zip(flat, [g for r in got for g in r]):
        if d[4] & 4:
            assert (g["n_contacts_x"], g["n_contacts_y"], g["n_contacts_xy"]) == orc.contacts_at_jamming(*d)
    assert st["requests_completed"] == len(MIX)
    assert st["samples_resident"] == 0 and st["arena_used"] == 0
    assert st["launches"] > 50   # the long samples were sliced


def test_time_sliced_long_kmers_with_slab_counts(ctx, orc):
    """Long k-mers (interval clear, compressed lattice) yielding and resuming
    at a 20 us quantum, with the interval clear's counts forced into the slab
    (two sets used by alternate steps, both cleared when a sample resumes)."""
    from paper_1810_06800_amd import rsa

    reqs = [[(1100, 512, 21, s, 0) for s in range(2)], [(1500, 700, 22, 0, 2)], [(2048, 600, 23, 1, 4)],
            [(600, 512, 24, 0, 0)]]
    ctx.set_option(rsa.OPT_IV_SLAB, 1)
    try:
        _log("server: long k-mers, counts in the slab, quantum 20 us")
        with rsa.Server(ctx, arena_bytes=1 << 30, quantum_us=20) as srv:
            got = srv.run(reqs)
            st = srv.stats()
    finally:
        ctx.set_option(rsa.OPT_IV_SLAB, 0)
    flat = [d for r in reqs for d in r]
    want = orc.run_many(flat, threads=min(16, os.cpu_count() or 1))
    same_as_oracle(flat, [g for r in got for g in r], want)
    for d, g in zip(flat, [g for r in got for g in r]):
        if d[4] & 4:
            assert (g["n_contacts_x"], g["n_contacts_y"], g["n_contacts_xy"]) == orc.contacts_at_jamming(*d)
    assert st["launches"] > 20   # the samples were sliced


def test_alone_and_in_the_mix_agree(ctx):
    """Each request gives the same results alone, in a mix that arrives while
    it runs, and through rsa_run_batch."""
    from paper_1810_06800_amd import rsa

    probe = [(1024, 64, 77, s, 2) for s in range(4)] + [(512, 128, 78, 0, 0)]
    batch = ctx.run(probe)
    with rsa.Server(ctx, arena_bytes=1 << 30, quantum_us=200) as srv:
        alone = srv.run([probe])[0]
    same(alone, batch)
    with rsa.Server(ctx, arena_bytes=1 << 30, quantum_us=200) as srv:
        rid = srv.submit(probe)
        others = []
        done = {}
        for step in range(100000):
            # new requests keep arriving while the probe is on the device
            if step < 12:
                others.append(srv.submit(MIX[step % len(MIX)]))
            srv.step(wait=True)
            for r in srv.completed():
                done[r] = srv.results(r)
            if len(done) == 1 + len(others) and step >= 12:
                break
        st = srv.stats()
    same(done[rid], batch)
    for i, r in enumerate(others):
        want = ctx.run(MIX[i % len(MIX)])
        same(done[r], want)
    assert st["requests_completed"] == 13


def test_admission_by_footprint(ctx, orc):
    """An arena that holds three (1024, 64) samples at a time: the rest queue
    and are admitted as slabs free up; a sample larger than the arena is
    refused at submission."""
    from paper_1810_06800_amd import rsa

    fp = rsa.footprint_bytes(1024, 64)
    arena = 3 * ((fp + 4095) // 4096 * 4096)
    reqs = [[(1024, 64, 20 + i, s, 0) for s in range(2)] for i in range(5)]
    with rsa.Server(ctx, arena_bytes=arena, quantum_us=500) as srv:
        with pytest.raises(rsa.RsaError) as e:
            srv.submit([(2048, 64, 0, 0, 0)])
        assert e.value.code == rsa.RSA_ENOMEM
        got = srv.run(reqs)
        st = srv.stats()
    assert st["arena_peak"] <= arena
    assert st["arena_peak"] >= 3 * fp
    flat = [d for r in reqs for d in r]
    same_as_oracle(flat, [g for r in got for g in r], orc.run_many(flat, threads=min(16, os.cpu_count() or 1)))


def test_resident_slot_cap(ctx):
    """max_resident = 2: at most two samples on the device at a time, all finish."""
    from paper_1810_06800_amd import rsa

    reqs = [[(64, 8, 1, s, 0) for s in range(5)], [(128, 16, 2, s, 0) for s in range(3)]]
    with rsa.Server(ctx, arena_bytes=1 << 28, quantum_us=100, max_resident=2) as srv:
        got = srv.run(reqs)
    for r, g in zip(reqs, got):
        same(g, ctx.run(r))


def test_invalid_requests_rejected(ctx):
    from paper_1810_06800_amd import rsa

    with rsa.Server(ctx, arena_bytes=1 << 26) as srv:
        for bad in [[(4, 5, 0, 0, 0)], [(16, 4, 0, 0, 32)], [(16, 4, 0, 0, 8)], []]:
            with pytest.raises(rsa.RsaError) as e:
                srv.submit(bad)
            assert e.value.code == rsa.RSA_EINVAL
        # still serves afterwards
        assert srv.run([[(8, 2, 0, 0, 0)]])[0][0]["status"] == 0
