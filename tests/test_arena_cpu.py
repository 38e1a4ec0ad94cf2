"""The request server's arena allocator (host code, csrc/arena.h), driven
through a small g++ build: ranges never overlap, stay aligned and inside the
arena, the byte accounting is exact, best fit is taken, and freeing
everything merges the free list back into one range."""
import os
import random
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ALIGN = 4096


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("arena") / "arena_driver")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-o", exe, os.path.join(HERE, "arena_driver.cpp")],
                   check=True)
    return exe


def run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
    return out.stdout.split("\n")[:-1]


def rnd(v):
    return (max(v, 1) + ALIGN - 1) // ALIGN * ALIGN


def test_random_alloc_free(driver):
    """600 random allocations and frees, offsets fed back from the driver's
    own answers (the script is replayed up to each allocation)."""
    rng = random.Random(5)
    size = 64 << 20
    assert run(driver, [f"reset {size}"]) == [f"size {size}"]
    cmds = [f"reset {size}"]
    live = {}
    used = 0
    for step in range(600):
        if live and rng.random() < 0.45:
            off = rng.choice(sorted(live))
            b = live.pop(off)
            cmds.append(f"free {off} {b}")
            used -= rnd(b)
        else:
            b = rng.choice([1, 100, 4096, 5000, 70000, 1 << 20, 3 << 20, 9 << 20])
            res = run(driver, cmds + [f"alloc {b}"])[-1]
            cmds.append(f"alloc {b}")
            if res == "full":
                # nothing fits: the largest free range is smaller than the request
                st = run(driver, cmds[:-1] + ["stat"])[-1].split()
                assert int(st[3]) < rnd(b)
                continue
            off = int(res.split()[1])
            assert off % ALIGN == 0 and off + rnd(b) <= size
            for o, ob in live.items():
                assert off + rnd(b) <= o or o + rnd(ob) <= off, "overlap"
            live[off] = b
            used += rnd(b)
        if step % 50 == 0:
            st = run(driver, cmds + ["stat"])[-1].split()
            assert int(st[1]) == used
    for off, b in list(live.items()):
        cmds.append(f"free {off} {b}")
    st = run(driver, cmds + ["stat"])[-1].split()
    assert st[1] == "0" and st[3:] == [str(size), "1"]


def test_best_fit_and_merge(driver):
    out = run(driver, ["reset 1000000", "alloc 4096", "alloc 8192", "alloc 4096", "alloc 16384",
                       "free 0 4096", "free 12288 4096", "alloc 4000", "stat"])
    assert out[0] == f"size {1000000 // ALIGN * ALIGN}"
    offs = [int(x.split()[1]) for x in out[1:5]]
    assert offs == [0, 4096, 12288, 16384]
    # two free holes of one page (0 and 12288) and the tail: best fit takes the first hole
    assert out[7] == "ok 0"
    out = run(driver, ["reset 65536", "alloc 16384", "alloc 16384", "alloc 16384", "free 16384 16384",
                       "free 0 16384", "free 32768 16384", "stat"])
    assert out[-1].split()[1:] == ["0", "49152", "65536", "1"]
    assert run(driver, ["reset 8192", "alloc 8193"])[-1] == "full"
