"""GPU parity: the HIP library, called through the C ABI, against the oracle.

Every field is an integer (counts, hashes, byte counts), so the bar is
bit-exact equality, sample by sample.  Shapes: every tiny torus (seams,
k = L, L <= 2), random shapes with ragged L % 64, H-only rings, the cluster
census, and the benchmark workloads at full size in the launch configuration
the benchmark times (all samples on the GPU, the oracle on all or a seeded
subset of them).
"""
import os
import random
import sys

import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("n_jam", "n_wrap_x", "n_wrap_y", "n_wrap_any", "occ_hash", "seq_hash",
          "alg_bytes", "wchg_words")


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


def check(descs, got, want, census=False):
    bad = []
    for d, g, w in zip(descs, got, want):
        assert w["status"] == 0, (d, w["status"])
        if g["status"] != 0:
            bad.append((d, "status", g["status"], 0))
            continue
        for f in FIELDS:
            if g[f] != w[f]:
                bad.append((d, f, g[f], w[f]))
                break
        if census and len(d) > 4 and d[4] & 2:
            if (g["n_clusters_jam"], g["n_nonwrapping_jam"]) != (w["n_clusters_jam"], 0):
                bad.append((d, "census", g["n_clusters_jam"], w["n_clusters_jam"]))
    assert not bad, f"{len(bad)} mismatches, first: {bad[:5]}"


def test_tiny_tori_every_k(ctx, orc):
    descs = []
    for L in range(1, 13):
        for k in range(1, L + 1):
            for seed, sample in ((0, 0), (0xDEADBEEFCAFEF00D, 12345)):
                descs.append((L, k, seed, sample, 2 if (L + k) % 2 else 0))
    _log(f"tiny tori: {len(descs)} samples")
    got = ctx.run(descs)
    check(descs, got, orc.run_many(descs), census=True)


def test_random_shapes(ctx, orc):
    rng = random.Random(99)
    descs = []
    for _ in range(200):
        L = rng.randint(2, 300)
        k = rng.randint(1, max(1, min(L, rng.choice([2, 4, 8, 16, 40, L]))))
        descs.append((L, k, rng.getrandbits(64), rng.getrandbits(32), rng.choice([0, 2])))
    _log(f"random shapes: {len(descs)} samples")
    got = ctx.run(descs)
    check(descs, got, orc.run_many(descs), census=True)


def test_h_only_rings(ctx, orc):
    descs = [(L, k, 5, s, 1) for L, k in [(64, 2), (48, 8), (33, 16), (130, 3)] for s in range(8)]
    got = ctx.run(descs)
    check(descs, got, orc.run_many(descs))


def test_plain_small_workload(ctx, orc):
    from paper_1810_06800_amd import workloads

    descs = workloads.plain_small()
    _log("plain_small: 256 x (64, 8)")
    got = ctx.run(descs)
    check(descs, got, orc.run_many(descs))


def test_plain_scale_workload_full(ctx, orc):
    """L = 1024, k = 64, seeds 0..1023: the benchmark's batch, all checked."""
    from paper_1810_06800_amd import workloads

    descs = workloads.plain_scale()
    _log("plain_scale: 1024 x (1024, 64)")
    got = ctx.run(descs)
    want = orc.run_many(descs, threads=min(16, os.cpu_count() or 1))
    check(descs, got, want)


def test_tiles_and_modes_agree(ctx, orc):
    """A sample's result does not depend on the schedule, the batch it sits in,
    or plain vs batched launches."""
    from paper_1810_06800_amd import rsa

    descs = [(64, 8, 1, s, 0) for s in range(4)] + [(200, 20, 3, 1, 2), (96, 96, 2, 0, 0),
                                                     (300, 7, 8, 2, 0), (130, 65, 4, 4, 2)]
    want = orc.run_many(descs)
    try:
        for tile in range(rsa.num_tiles()):
            ctx.set_option(rsa.OPT_TILE, tile)
            got = ctx.run(descs)
            check(descs, got, want, census=True)
            assert all(g["tile"] == tile for g in got)
        ctx.set_option(rsa.OPT_TILE, -1)
        ctx.set_option(rsa.OPT_MODE, rsa.MODE_PLAIN)
        check(descs, ctx.run(descs), want, census=True)
        ctx.set_option(rsa.OPT_MODE, rsa.MODE_BATCHED)
        ctx.set_option(rsa.OPT_GRAPH, 0)
        check(descs, ctx.run(descs), want, census=True)
        ctx.set_option(rsa.OPT_GRAPH, 1)
        ctx.set_option(rsa.OPT_SLOTS, 3)
        mixed = descs + [(128, 4, 9, s, 0) for s in range(20)]
        got = ctx.run(mixed)
        check(descs, got[: len(descs)], want, census=True)
        # alone vs in the mix
        for i in (0, 5):
            check([descs[i]], ctx.run([descs[i]]), [want[i]], census=True)
    finally:
        ctx.set_option(rsa.OPT_TILE, -1)
        ctx.set_option(rsa.OPT_MODE, rsa.MODE_BATCHED)
        ctx.set_option(rsa.OPT_GRAPH, 1)
        ctx.set_option(rsa.OPT_SLOTS, 0)


def test_results_as_array(ctx):
    """The structured-array view of a batch's results equals the dicts."""
    descs = [(64, 8, 5, s, 0) for s in range(6)]
    want = ctx.run(descs)
    arr = ctx.results(ctx.run_batch(descs), as_array=True)
    assert len(arr) == len(want)
    for r, w in zip(arr, want):
        assert {f: r[f].item() for f in arr.dtype.names} == w


def test_graph_replays_repeat(ctx, orc):
    """The same batch replayed from the cached graph gives the same results,
    with other work and synchronisations in between."""
    import torch

    descs = [(100, 10, 11, s, 0) for s in range(12)]
    want = orc.run_many(descs)
    for rep in range(4):
        check(descs, ctx.run(descs), want)
        x = torch.ones(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert float(x.sum()) == float(1 << 20)


def test_wide_rows(ctx, orc):
    """Rows of more than 64 bitmap words (L > 4096) use the wide kernels."""
    descs = [(4160, 64, 7, s, 0) for s in range(3)] + [(4097, 300, 1, 0, 2)]
    _log("wide rows: (4160, 64) x 3, (4097, 300)")
    got = ctx.run(descs)
    check(descs, got, orc.run_many(descs), census=True)


def test_mixed_batch_workload(ctx, orc):
    """The uneven batch: 512 samples over five (L, k) shapes in one graph,
    every sample against the oracle."""
    from paper_1810_06800_amd import workloads

    descs = workloads.mixed_batch()
    _log("mixed batch: 512 samples")
    got = ctx.run(descs)
    assert all(g["status"] == 0 for g in got)
    _log("mixed batch: oracle on all 512")
    check(descs, got, orc.run_many(descs, threads=min(16, os.cpu_count() or 1)))


def test_large_workloads_every_sample(ctx):
    """L = 16384, k = 1024 (32 samples) and L = 32768, k = 4096 (8 samples) at
    full size, each as one batch as the benchmark launches it; every sample
    against the oracle's stored results (tests/golden/make_large_expected.py)
    and the proven bounds."""
    import json

    from paper_1810_06800_amd import workloads

    with open(os.path.join(os.path.dirname(__file__), "golden", "large_expected.json")) as f:
        golden = json.load(f)
    want = {tuple(d): r for d, r in zip(golden["descs"], golden["results"])}
    for name in ("large_16k", "large_32k"):
        descs = workloads.CONFIGS[name]()
        _log(f"{name}: {len(descs)} samples")
        got = ctx.run(descs)
        for d, g in zip(descs, got):
            L, k = d[0], d[1]
            assert g["status"] == 0, (d, g["status"])
            assert 1 <= g["n_wrap_any"] <= g["n_jam"] and g["n_jam"] * k <= L * L
        assert all(tuple(d) in want for d in descs)
        check(descs, got, [want[tuple(d)] for d in descs])


def test_autotune_table_applied(ctx, orc):
    """Shapes in the autotune table run with the table's tile, others with the
    heuristic, and results match the oracle either way."""
    from paper_1810_06800_amd import rsa

    table = {(L, k): t for L, k, t in rsa.load_tile_table()}
    assert table
    descs = [(2048, 128, 5, 0, 0), (512, 32, 5, 1, 0), (300, 7, 5, 2, 0)]
    got = ctx.run(descs)
    for d, g in zip(descs, got):
        want_tile = table.get(d[:2], rsa.tile_for_shape(d[0], d[1]))
        assert g["tile"] == want_tile == ctx.tile_for_sample(d[0], d[1])
    check(descs, got, orc.run_many(descs))
    with pytest.raises(rsa.RsaError):
        ctx.set_tile_table([(4, 8, 0)])
    assert ctx.tile_for_sample(2048, 128) == table[(2048, 128)]   # table unchanged


def test_contact_census(ctx, orc):
    """RSA_FLAG_CONTACTS: the census of the jammed state (Eq. 12) against the
    oracle's, on tiny tori, ragged and wide lattices, rings and one full
    L = 1024, k = 64 sample; the other fields are unchanged by the flag."""
    from paper_1810_06800_amd import rsa

    descs = [(L, k, 3, s, 4) for L in (1, 2, 3, 5, 8) for k in range(1, L + 1) for s in range(2)]
    descs += [(64, 8, 1, s, 4) for s in range(4)] + [(200, 20, 3, 1, 6), (130, 65, 4, 4, 4),
                                                      (96, 4, 9, 0, 5), (300, 7, 8, 2, 4),
                                                      (4160, 64, 7, 0, 4), (1024, 64, 2, 0, 4)]
    _log(f"contact census: {len(descs)} samples")
    got = ctx.run(descs)
    check(descs, got, orc.run_many(descs, threads=min(16, os.cpu_count() or 1)), census=True)
    for d, g in zip(descs, got):
        want = orc.contacts_at_jamming(*d)
        assert (g["n_contacts_x"], g["n_contacts_y"], g["n_contacts_xy"]) == want, d
    plain = ctx.run([d[:4] + (d[4] & ~rsa.FLAG_CONTACTS,) for d in descs[-3:]])
    for g, p in zip(got[-3:], plain):
        assert p["n_contacts_x"] == -1
        assert all(g[f] == p[f] for f in FIELDS)


def size_bins(exact):
    """The oracle's exact histogram (index = cluster size in sites) in
    power-of-two bins: bin b holds sizes 2^b .. 2^(b+1)-1."""
    out = [0] * 32
    for size, count in enumerate(exact):
        if count:
            out[size.bit_length() - 1] += count
    return out


def test_cluster_sizes_at_first_wrap(ctx, orc):
    """RSA_FLAG_CLUSTER_SIZES: the histogram of cluster sizes right after
    deposit n_wrap_any (Eq. 11) against the oracle's snapshot at that step,
    in the batched, plain and graph-less forms; other samples read zero and
    every result is unchanged by the flag."""
    from paper_1810_06800_amd import rsa

    descs = [(L, k, 7, s, 8) for L in (1, 2, 3, 4, 6, 9) for k in range(1, L + 1) for s in range(2)]
    descs += [(64, 8, 1, s, 8) for s in range(3)] + [(200, 20, 3, 1, 10), (130, 65, 4, 4, 12),
                                                      (300, 7, 8, 2, 8), (96, 4, 9, 0, 0),
                                                      (1024, 64, 2, 0, 8), (1100, 512, 6, 0, 8)]
    _log(f"cluster sizes: {len(descs)} samples")
    want = orc.run_many([d[:4] + (d[4] & 7,) for d in descs], threads=min(16, os.cpu_count() or 1))
    exact = [size_bins(orc.run(*d[:4], flags=d[4] & 7, snap_step=w["n_wrap_any"],
                               snap_cap=d[0] * d[0] + 1)["snap_hist"]) if d[4] & 8 else [0] * 32
             for d, w in zip(descs, want)]
    try:
        for mode, graph in ((rsa.MODE_BATCHED, 1), (rsa.MODE_PLAIN, 1), (rsa.MODE_BATCHED, 0)):
            ctx.set_option(rsa.OPT_MODE, mode)
            ctx.set_option(rsa.OPT_GRAPH, graph)
            b = ctx.run_batch(descs)
            hist = ctx.cluster_sizes(b)
            got = ctx.results(b)
            check(descs, got, want, census=True)
            bad = [(d, h, e) for d, h, e in zip(descs, hist, exact) if h != e]
            assert not bad, f"{len(bad)} histograms differ, first {bad[0]}"
    finally:
        ctx.set_option(rsa.OPT_MODE, rsa.MODE_BATCHED)
        ctx.set_option(rsa.OPT_GRAPH, 1)
    # a batch without the flag has no histograms
    b = ctx.run_batch([(64, 8, 1, 0, 0)])
    with pytest.raises(rsa.RsaError):
        ctx.cluster_sizes(b)
    ctx.results(b)


def test_invalid_descriptors_rejected(ctx):
    from paper_1810_06800_amd import rsa

    for bad in [(4, 5, 0, 0, 0), (0, 0, 0, 0, 0), (32769, 8, 0, 0, 0), (16, 4, 0, 0, 16), (16, 4, 0, 0, 32)]:
        with pytest.raises(rsa.RsaError) as e:
            ctx.run_batch([bad])
        assert e.value.code == rsa.RSA_EINVAL
    # the context still works afterwards
    assert ctx.run([(8, 2, 0, 0, 0)])[0]["status"] == 0
    assert ctx.run([]) == []


def test_library_loaded_before_torch(orc):
    """A process that loads the library before it imports torch still gets a
    working context (one HIP runtime in the process), with exact results."""
    import subprocess

    code = ("from paper_1810_06800_amd import rsa\n"
            "rsa.lib()\n"
            "ctx = rsa.Context(0)\n"
            "r = ctx.run([(24, 3, 11, 2, 0)])[0]\n"
            "print('result', r['n_jam'], r['occ_hash'], r['n_wrap_any'], flush=True)\n"
            "ctx.close()\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=240)
    assert out.returncode == 0, out.stderr[-3000:]
    want = orc.run(24, 3, 11, 2, 0)
    line = [l for l in out.stdout.splitlines() if l.startswith("result")][0]
    assert line.split()[1:] == [str(want["n_jam"]), str(want["occ_hash"]), str(want["n_wrap_any"])]


def test_all_statistics_together(ctx, orc):
    """Cluster census, contact census and cluster sizes requested together
    (flags 2 | 4 | 8) at the benchmark shape and a smaller one: every figure
    matches the oracle's, and the counts are those of the flagless run."""
    descs = [(1024, 64, 21, s, 14) for s in range(4)] + [(512, 32, 22, s, 14) for s in range(4)]
    _log(f"all statistics: {len(descs)} samples")
    want = orc.run_many([d[:4] + (d[4] & 7,) for d in descs], threads=min(16, os.cpu_count() or 1))
    b = ctx.run_batch(descs)
    hist = ctx.cluster_sizes(b)
    got = ctx.results(b)
    check(descs, got, want, census=True)
    for d, g, w, h in zip(descs, got, want, hist):
        assert (g["n_contacts_x"], g["n_contacts_y"], g["n_contacts_xy"]) == orc.contacts_at_jamming(*d[:4], 6), d
        snap = orc.run(*d[:4], flags=6, snap_step=w["n_wrap_any"], snap_cap=d[0] * d[0] + 1)["snap_hist"]
        assert h == size_bins(snap), d
    plain = ctx.run([d[:4] + (0,) for d in descs])
    for g, p in zip(got, plain):
        assert all(g[f] == p[f] for f in FIELDS)


def test_full_ring_kmers_at_the_row_width_limit(ctx, orc):
    """k = L on both sides of the one-wave row limit (L = 4096 and 4097):
    every deposit covers a whole ring, the first one wraps in its own
    direction and the other direction wraps only at jamming (n = L)."""
    descs = [(4096, 4096, 5, 0, 2), (4096, 4096, 5, 1, 2), (4097, 4097, 5, 0, 2)]
    _log(f"k = L at the row-width limit: {descs}")
    want = [orc.run(*d) for d in descs]
    got = ctx.run(descs)
    check(descs, got, want, census=True)
    for d, g in zip(descs, got):
        assert g["n_jam"] == d[0] and g["n_wrap_any"] == 1
        assert max(g["n_wrap_x"], g["n_wrap_y"]) == d[0]


def test_long_kmers_interval_clear_and_compressed_lattice(ctx, orc):
    """Long k-mers (k >= 512): the interval clear (anchor-interval buckets) and
    the compressed lattice (occupancy and anchor bitmaps with the placement
    table instead of the site map), on narrow and wide rows, ragged L % 64,
    k = L, k near L/2, with every statistic flag, under every selecting-wave
    count; and the summary-bit clear where the interval one does not apply
    (k > 4096)."""
    from paper_1810_06800_amd import rsa

    descs = [(512, 512, 3, 0, 0), (600, 512, 3, 1, 2), (1000, 513, 4, 0, 4), (1024, 600, 4, 1, 0),
             (1500, 700, 5, 0, 6), (2048, 512, 5, 1, 0), (2999, 1499, 6, 0, 2), (4100, 1025, 6, 1, 4),
             (4097, 2100, 7, 0, 0), (5000, 2600, 7, 1, 2), (8192, 4097, 8, 0, 6)]
    descs += [(1100, 550, 9, s, 0) for s in range(6)]
    want = orc.run_many(descs, threads=min(16, os.cpu_count() or 1))
    _log(f"long k-mers: {len(descs)} samples, default tiles")
    got = ctx.run(descs)
    check(descs, got, want, census=True)
    for d, g, w in zip(descs, got, want):
        if d[4] & 4:
            assert (g["n_contacts_x"], g["n_contacts_y"], g["n_contacts_xy"]) == \
                orc.contacts_at_jamming(*d[:4]), d
    try:
        for waves in range(5):
            tile = rsa.tile_for_shape(1024, 600)
            w0, tr, mr, sp = rsa.tile_shape(tile)
            # same bitmap / map tiles and clear mode, each wave count
            t = next(t for t in range(rsa.num_tiles())
                     if rsa.tile_shape(t) == ((1, 2, 3, 7, 15)[waves], tr, mr, sp))
            ctx.set_option(rsa.OPT_TILE, t)
            sub = descs[:8]
            _log(f"long k-mers: tile {t} ({rsa.tile_shape(t)})")
            check(sub, ctx.run(sub), want[:8], census=True)
    finally:
        ctx.set_option(rsa.OPT_TILE, -1)


def test_interval_counts_in_the_slab(ctx, orc):
    """The interval clear with its difference counts in the slab, in two sets
    used by alternate steps (the layout L = 32768 needs), forced on shapes
    whose counts would fit LDS: narrow and wide rows, ragged L % 64, k = L,
    k near L/2, every statistic flag, several selecting-wave counts, and
    samples of L = 16384, k = 1024 against the stored oracle results."""
    import json

    from paper_1810_06800_amd import rsa

    descs = [(512, 512, 3, 0, 0), (600, 512, 3, 1, 2), (1000, 513, 4, 0, 4), (1024, 600, 4, 1, 0),
             (1500, 700, 5, 0, 6), (2048, 512, 5, 1, 0), (2999, 1499, 6, 0, 2), (4100, 1025, 6, 1, 4)]
    descs += [(1100, 550, 9, s, 0) for s in range(4)]
    want = orc.run_many(descs, threads=min(16, os.cpu_count() or 1))
    with open(os.path.join(os.path.dirname(__file__), "golden", "large_expected.json")) as f:
        golden = json.load(f)
    big = [tuple(d) for d in golden["descs"] if d[0] == 16384][:4]
    big_want = {tuple(d): r for d, r in zip(golden["descs"], golden["results"])}
    ctx.set_option(rsa.OPT_IV_SLAB, 1)
    try:
        assert ctx.get_option(rsa.OPT_IV_SLAB) == 1
        _log(f"interval counts in the slab: {len(descs)} samples, default tiles")
        check(descs, ctx.run(descs), want, census=True)
        _log(f"interval counts in the slab: {len(big)} samples of L = 16384")
        check(big, ctx.run(big), [big_want[d] for d in big])
        for waves in (1, 2, 7):
            tile = rsa.tile_for_shape(1024, 600)
            w0, tr, mr, sp = rsa.tile_shape(tile)
            t = next(t for t in range(rsa.num_tiles()) if rsa.tile_shape(t) == (waves, tr, mr, sp))
            ctx.set_option(rsa.OPT_TILE, t)
            _log(f"interval counts in the slab: tile {t} ({rsa.tile_shape(t)})")
            check(descs[:6], ctx.run(descs[:6]), want[:6], census=True)
    finally:
        ctx.set_option(rsa.OPT_TILE, -1)
        ctx.set_option(rsa.OPT_IV_SLAB, 0)


def test_small_budget_reuses_slabs(orc):
    """A context whose memory budget holds only a few slabs runs a larger
    batch with a few workgroups, each taking sample after sample on the same
    slab (every sample re-initialised), with exact results."""
    from paper_1810_06800_amd import rsa

    descs = [(256, 8, 31, s, 0) for s in range(40)] + [(300, 5, 32, s, 2) for s in range(8)]
    foot = max(rsa.footprint_bytes(256, 8), rsa.footprint_bytes(300, 5))
    small = rsa.Context(0, budget_bytes=6 * foot + (8 << 20))
    try:
        _log(f"small budget: {len(descs)} samples, budget {6 * foot + (8 << 20)} B")
        got = small.run(descs)
    finally:
        small.close()
    check(descs, got, orc.run_many(descs, threads=min(16, os.cpu_count() or 1)), census=True)
