"""The host C/C++ code under AddressSanitizer and UBSan: the oracle (run,
sequence capture, cluster-size histogram, contact census) and the request
server's arena allocator, built with gcc/g++ -fsanitize=address,undefined and
driven through edge cases (L = k, k = 1, L = 1, one-dimensional rings, a
sequence buffer that is too small, rejected descriptors).  Any sanitizer
report fails the test (halt_on_error), and the sanitized oracle must print the
same numbers as the ordinary build."""
import os
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")

# (L, k, seed, sample, flags, snap_step, seq_cap)
CASES = [
    (1, 1, 3, 0, 0, 1, 4),           # one site
    (2, 2, 5, 1, 0, 1, 8),           # k = L: a k-mer covers a whole ring
    (7, 7, 11, 2, 0, 1, 64),
    (9, 1, 13, 0, 0, 40, 200),       # monomers: fills the torus
    (37, 5, 17, 3, 0, 30, 1000),     # ragged word tails
    (64, 8, 19, 0, 0, 50, 1000),
    (65, 3, 23, 4, 2, 100, 2000),    # cluster census flag
    (33, 4, 29, 0, 1, 5, 400),       # one-dimensional rings
    (48, 6, 31, 5, 4, 20, 2),        # sequence buffer too small
    (0, 1, 1, 0, 0, 0, 0),           # rejected: L = 0 (k > L)
    (8, 9, 1, 0, 0, 0, 0),           # rejected: k > L
    (8, 2, 1, 0, 16, 0, 0),          # rejected: unknown flag
]


@pytest.fixture(scope="module")
def oracle_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "oracle_san")
    subprocess.run(["gcc", *SAN, "-std=c11", "-o", exe, os.path.join(HERE, "sanitize_driver.c"),
                    os.path.join(ROOT, "oracle", "rsa_oracle.c"), "-lm"], check=True)
    return exe


def test_oracle_clean_under_sanitizers(oracle_exe):
    inp = "".join(" ".join(str(v) for v in c) + "\n" for c in CASES)
    out = subprocess.run([oracle_exe], input=inp, capture_output=True, text=True, env=ENV, timeout=300)
    assert out.returncode == 0, out.stderr[-3000:]
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr[-3000:]
    lines = out.stdout.strip().split("\n")
    assert len(lines) == len(CASES)
    for case, line in zip(CASES, lines):
        L, k, seed, sample, flags, snap, cap = case
        v = [int(x) for x in line.split()]
        rc = v[0]
        if k < 1 or k > L or flags & ~7:
            assert rc == -1 and v[11] == -1, case
            continue
        ref = oracle.run(L, k, seed, sample, flags)
        if cap and cap < ref["n_jam"]:
            assert rc == -14, case        # the caller's sequence buffer was too small
        else:
            assert rc == 0, case
            assert v[1:11] == [ref["n_jam"], ref["n_wrap_x"], ref["n_wrap_y"], ref["n_wrap_any"],
                               ref["occ_hash"], ref["seq_hash"], ref["n_clusters_jam"],
                               ref["n_nonwrapping_jam"], ref["alg_bytes"], ref["wchg_words"]], case
        assert v[11] == 0, case
        assert tuple(v[12:15]) == tuple(oracle.contacts_at_jamming(L, k, seed, sample, flags)), case


@pytest.fixture(scope="module")
def arena_exe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "arena_san")
    subprocess.run(["g++", *SAN, "-std=c++17", "-o", exe, os.path.join(HERE, "arena_driver.cpp")], check=True)
    return exe


def test_arena_clean_under_sanitizers(arena_exe):
    import random

    rng = random.Random(9)
    sizes = [1, 4095, 4096, 4097, 1 << 16, 5 << 20, 40 << 20]
    pending = [f"alloc {rng.choice(sizes)}" for _ in range(1500)]
    script, live = [f"reset {256 << 20}"], []
    # drive allocation and release in chunks so frees name real offsets
    for chunk in range(0, len(pending), 50):
        batch = pending[chunk:chunk + 50]
        out = subprocess.run([arena_exe], input="\n".join(script + batch) + "\n", capture_output=True,
                             text=True, env=ENV, timeout=120)
        assert out.returncode == 0, out.stderr[-3000:]
        got = out.stdout.strip().split("\n")[-len(batch):]
        for c, g in zip(batch, got):
            if g.startswith("ok"):
                live.append((int(g.split()[1]), int(c.split()[1])))
        script += batch
        for _ in range(len(live) // 2):
            off, b = live.pop(rng.randrange(len(live)))
            script.append(f"free {off} {b}")
        script.append("stat")
    for off, b in live:
        script.append(f"free {off} {b}")
    script.append("stat")
    out = subprocess.run([arena_exe], input="\n".join(script) + "\n", capture_output=True, text=True,
                         env=ENV, timeout=120)
    assert out.returncode == 0, out.stderr[-3000:]
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr
    used, peak, largest, ranges = (int(x) for x in out.stdout.strip().split("\n")[-1].split()[1:])
    assert used == 0 and largest == 256 << 20 and ranges == 1 and peak > 0
