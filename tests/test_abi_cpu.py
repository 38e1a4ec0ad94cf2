"""The C-ABI library loads on the CPU and exports what include/rsa.h declares.

No compute call is made: only entry points that need no device.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsa.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsa_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def rsa():
    from paper_1810_06800_amd import rsa as mod

    if not os.path.exists(mod.LIB_PATH):
        pytest.fail("librsa_hip.so not built: run __graft_entry__.build()")
    return mod


def test_every_declared_symbol_is_exported(rsa):
    lib = rsa.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(rsa.EXPORTS)


def test_record_layouts(rsa):
    import ctypes

    assert ctypes.sizeof(rsa.Sample) == 24
    assert ctypes.sizeof(rsa.Result) == 104
    assert ctypes.sizeof(rsa.ServerConfig) == 16


def test_footprint_matches_layout(rsa):
    # two bitmaps of L*ceil(L/64) words, int32 map, 20 B per k-mer record,
    # every area 256-byte aligned
    # (rows and columns padded so that every 128-byte tile shape fits),
    # plus a 256-byte state record and room for the 2L uint16 row counts and
    # their sums over 64 and 4096 rows (time-sliced runs), and when a line has
    # at most 64 buckets of k+1 positions, the anchor-interval buckets of the
    # H rows and of the V columns (4 B per bucket and line)
    def expect(L, k):
        a = lambda v: (v + 255) // 256 * 256
        r16 = lambda v: (v + 15) // 16 * 16
        wp = ((L + 63) // 64 + 15) // 16 * 16
        lp = (L + 31) // 32 * 32
        cap = L * L // k + 1
        summary = a(lp * ((wp + 63) // 64) * 8)
        rows = 2 * L
        counts = r16((rows + 1) // 2 * 4) + r16((rows + 63) // 64 * 4) + r16((rows + 4095) // 4096 * 4)
        nb = (L + k) // (k + 1)
        buckets = 2 * a(4 * nb * lp) if nb <= 64 else 0
        # long k-mers (k >= 512, the sparse-clear tiles the heuristic picks)
        # keep six one-bit-per-site bitmaps and a placement table of a power
        # of two >= 2 (L^2/k + 1) 8-byte slots instead of the int32 map
        compressed = k >= 512
        site_map = 0 if compressed else a(4 * lp * lp)
        slots = 64
        while slots < 2 * (L * L // k + 1):
            slots *= 2
        bitmaps = 6 * a(((L + 63) // 64) * ((L + 15) // 16) * 16 * 8) + a(8 * slots) if compressed else 0
        # shapes the interval clear takes (k <= 4096, buckets): two sets of its
        # k + 1 difference counts (rounded to 4) and 68 sums, for lattices
        # whose LDS cannot hold them
        diffs = 2 * 4 * (((k + 1 + 3) // 4) * 4 + 68) if (k <= 4096 and nb <= 64) else 0
        return (a(lp * wp * 8) * 2 + summary * 2 + site_map + a(16 * cap) + a(4 * cap)
                + a(256 + counts) + buckets + bitmaps + a(diffs))

    for L, k in [(1, 1), (5, 3), (64, 8), (1024, 64), (16384, 1024), (32768, 4096), (16384, 2),
                 (130, 1), (4096, 63), (4097, 4097), (600, 512), (1000, 511)]:
        assert rsa.footprint_bytes(L, k) == expect(L, k)
    assert rsa.footprint_bytes(1024, 64) < 5 * 2**20
    # the compressed lattice: one byte per site at L = 32768, k = 4096 (two
    # availability and six lattice bits), down from 4.3 GiB with the int32 map
    assert 1.0 * 2**30 < rsa.footprint_bytes(32768, 4096) < 1.1 * 2**30
    assert rsa.footprint_bytes(16384, 1024) < 0.3 * 2**30
    for L, k in [(0, 0), (4, 5), (32769, 8), (8, 0)]:
        assert rsa.footprint_bytes(L, k) == 0


def test_strerror_and_tiles(rsa):
    for code in range(-6, 1):
        assert rsa.strerror(code) and rsa.strerror(code) != "unknown status"
    assert rsa.strerror(-99) == "unknown status"
    n = rsa.num_tiles()
    assert n >= 1
    for L, k in [(64, 8), (1024, 64), (4096, 256), (16384, 1024), (32768, 4096)]:
        assert 0 <= rsa.tile_for_shape(L, k) < n
    assert rsa.tile_for_shape(4, 5) == rsa.RSA_EINVAL
    shapes = {rsa.tile_shape(t) for t in range(n)}
    assert len(shapes) == n
    for waves, tr, mr, sparse in shapes:
        assert 1 <= waves <= 15 and tr in (1, 2, 4, 8, 16) and mr in (1, 2, 4, 8, 16, 32)
        assert sparse in (0, 1)
        assert 64 * (waves + 1) <= 1024
    with pytest.raises(rsa.RsaError):
        rsa.tile_shape(n)


def test_workloads_shapes():
    from paper_1810_06800_amd import workloads as w

    assert len(w.plain_small()) == 256 and all(d[:2] == (64, 8) for d in w.plain_small())
    assert len(w.plain_scale()) == 1024 and {d[2] for d in w.plain_scale()} == set(range(1024))
    mixed = w.mixed_batch()
    assert len(mixed) == 512 and {d[:2] for d in mixed} == set(w.MIXED_SHAPES)
    assert mixed == w.mixed_batch()  # seeded
    assert len(w.large_16k()) == 32 and len(w.large_32k()) == 8
    tr = w.serving_trace(200)
    assert all(2 <= r["k"] <= r["L"] // 8 and 1 <= r["n"] <= 64 for r in tr)
    gaps = [b["arrival_s"] - a["arrival_s"] for a, b in zip(tr, tr[1:])]
    assert 0.003 < sum(gaps) / len(gaps) < 0.008


def test_autotune_table_is_well_formed(rsa):
    """The committed autotune table names valid shapes and tiles, each the
    fastest of the tiles it records for its shape."""
    import json

    with open(rsa.TILE_TABLE) as f:
        t = json.load(f)
    assert t["entries"]
    n = rsa.num_tiles()
    for e in t["entries"]:
        assert 1 <= e["k"] <= e["L"] <= 32768
        assert 0 <= e["tile"] < n
        tried = {int(k): v for k, v in e["tried"].items()}
        assert e["tile"] in tried and e["heuristic_tile"] in tried
        # the table's tile is the heuristic's unless another was clearly faster
        assert tried[e["tile"]] <= tried[e["heuristic_tile"]]
        assert tried[e["tile"]] <= min(tried.values()) * 1.05
        assert rsa.tile_shape(e["tile"])[0] in (1, 2, 3, 7)
    assert [(L, k, tile) for L, k, tile in rsa.load_tile_table()] == [
        (e["L"], e["k"], e["tile"]) for e in t["entries"]]


def test_missing_library_fails_loudly():
    """Without the built library the binding raises; there is no fallback."""
    import subprocess
    import sys

    code = ("import paper_1810_06800_amd.rsa as r\n"
            "r.LIB_PATH = '/nonexistent/librsa_hip.so'\n"
            "r._lib = None\n"
            "try:\n"
            "    r.Context(0)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "raised:" in out.stdout and "missing" in out.stdout


def test_static_scratch_constants(rsa):
    text = open(HEADER).read()
    m = re.search(r"#define RSA_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == rsa.STATIC_SCRATCH_BYTES
    m = re.search(r"#define RSA_STATIC_MAX_SAMPLES (\d+)", text)
    assert m and int(m.group(1)) == rsa.STATIC_MAX_SAMPLES
