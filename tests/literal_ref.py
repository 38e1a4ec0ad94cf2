"""Literal reference for one RSA run on an L x L torus (arXiv:1810.06800).

Test tool, independent of both the C oracle and the GPU library.  Everything
is recomputed from scratch after every deposit, straight from the definition:

* the available placements are found by testing all 2*L*L (o, y, x) for k
  empty sites (Sec. II.B "viable" placements), listed in canonical order
  P = o*L*L + y*L + x;
* the placement of rank floor(u * A / 2^64) is taken, u from Philox4x32-10
  keyed by the seed with counter (t, sample, 0, 0);
* wrapping is found by a breadth-first search of every cluster of occupied
  sites that assigns unwrapped coordinates; an edge whose two ends disagree
  with their unwrapped offset closes a cycle that winds round the torus
  (Sec. II.D, Newman-Ziff style).

The full run with windings is only for tiny lattices (L <= 12 or so); the
availability-only and 2k-test runs reach L of a few hundred.
"""
from __future__ import annotations

from collections import deque

import numpy as np

MASK32 = 0xFFFFFFFF
MASK64 = 0xFFFFFFFFFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) on Python integers."""
    x0, x1, x2, x3 = ctr
    k0, k1 = key
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & MASK32
            k1 = (k1 + 0xBB67AE85) & MASK32
        p0 = 0xD2511F53 * x0
        p1 = 0xCD9E8D57 * x2
        x0, x1, x2, x3 = ((p1 >> 32) ^ x1 ^ k0, p1 & MASK32, (p0 >> 32) ^ x3 ^ k1, p0 & MASK32)
    return x0, x1, x2, x3


def mix64(z: int) -> int:
    """SplitMix64 finalizer (Steele, Lea, Flood 2014)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def draw_u(seed: int, sample: int, t: int) -> int:
    r = philox4x32_10((t & MASK32, sample & MASK32, 0, 0), (seed & MASK32, (seed >> 32) & MASK32))
    return r[0] | (r[1] << 32)


def available(occ: np.ndarray, k: int, h_only: bool = False) -> list[int]:
    """Canonical indices of every placement whose k sites are all empty."""
    L = occ.shape[0]
    free = ~occ
    fits_h = np.ones((L, L), dtype=bool)
    fits_v = np.ones((L, L), dtype=bool)
    for i in range(k):
        fits_h &= np.roll(free, -i, axis=1)  # site (y, x+i)
        fits_v &= np.roll(free, -i, axis=0)  # site (y+i, x)
    if h_only:
        fits_v[:] = False
    idx = list(np.flatnonzero(fits_h.ravel()))
    idx += [L * L + int(i) for i in np.flatnonzero(fits_v.ravel())]
    return [int(i) for i in idx]


def clusters_and_windings(occ: np.ndarray):
    """Label clusters of occupied sites (4-neighbour adjacency on the torus)
    and report, per cluster, whether some closed path winds in x / in y."""
    L = occ.shape[0]
    label = -np.ones((L, L), dtype=np.int64)
    pos = {}
    out = []
    for sy in range(L):
        for sx in range(L):
            if not occ[sy, sx] or label[sy, sx] >= 0:
                continue
            c = len(out)
            wx = wy = False
            label[sy, sx] = c
            pos[(sy, sx)] = (sx, sy)
            q = deque([(sy, sx)])
            size = 0
            while q:
                y, x = q.popleft()
                size += 1
                ux, uy = pos[(y, x)]
                for ex, ey in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    ny, nx = (y + ey) % L, (x + ex) % L
                    if not occ[ny, nx]:
                        continue
                    want = (ux + ex, uy + ey)
                    if label[ny, nx] < 0:
                        label[ny, nx] = c
                        pos[(ny, nx)] = want
                        q.append((ny, nx))
                    else:
                        have = pos[(ny, nx)]
                        if have[0] != want[0]:
                            wx = True
                        if have[1] != want[1]:
                            wy = True
            out.append((size, wx, wy))
    return label, out


def contacts(owner: np.ndarray, orient: list[int]) -> tuple[int, int, int]:
    """(n_x, n_y, n_xy) of a configuration (Eq. 12): for every site, its right
    and its lower neighbour; a pair of occupied sites in different k-mers
    counts for both-horizontal, both-vertical or perpendicular."""
    L = owner.shape[0]
    out = [0, 0, 0]
    for y in range(L):
        for x in range(L):
            a = owner[y, x]
            if a < 0:
                continue
            for ny, nx in ((y, (x + 1) % L), ((y + 1) % L, x)):
                b = owner[ny, nx]
                if b < 0 or b == a:
                    continue
                oa, ob = orient[a], orient[b]
                out[2 if oa != ob else oa] += 1
    return tuple(out)


def size_histogram(occ: np.ndarray) -> dict[int, int]:
    """{cluster size in sites: number of clusters} of a configuration."""
    hist = {}
    for size, _, _ in clusters_and_windings(occ)[1]:
        hist[size] = hist.get(size, 0) + 1
    return hist


def run(L: int, k: int, seed: int, sample: int, h_only: bool = False, snap_step: int = 0) -> dict:
    """One run to jamming.  Besides the result fields: ``owner`` (final site ->
    deposit number grid), ``orient`` (per deposit, 0 = H, 1 = V) and, for
    snap_step > 0, ``snap_hist`` (cluster sizes right after that deposit)."""
    occ = np.zeros((L, L), dtype=bool)
    owner = -np.ones((L, L), dtype=np.int64)
    orient = []
    snap_hist = None
    seq = []
    n_x = n_y = -1
    seq_hash = 0
    t = 0
    while True:
        av = available(occ, k, h_only)
        A = len(av)
        if A == 0:
            break
        u = draw_u(seed, sample, t)
        rank = (u * A) >> 64
        P = av[rank]
        seq.append(P)
        seq_hash = (seq_hash + mix64((t << 32) | P)) & MASK64
        o, rem = divmod(P, L * L)
        y, x = divmod(rem, L)
        for i in range(k):
            sy, sx = ((y + i) % L, x) if o else (y, (x + i) % L)
            assert not occ[sy, sx]
            occ[sy, sx] = True
            owner[sy, sx] = t
        orient.append(o)
        _, cl = clusters_and_windings(occ)
        if snap_step and t + 1 == snap_step:
            snap_hist = size_histogram(occ)
        if n_x < 0 and any(c[1] for c in cl):
            n_x = t + 1
        if n_y < 0 and any(c[2] for c in cl):
            n_y = t + 1
        t += 1
    _, cl = clusters_and_windings(occ)
    defined = [v for v in (n_x, n_y) if v > 0]
    occ_hash = 0
    for s in np.flatnonzero(owner.ravel() >= 0):
        occ_hash = (occ_hash + mix64((int(s) << 32) | int(owner.ravel()[s]))) & MASK64
    return {
        "n_jam": t,
        "n_wrap_x": n_x,
        "n_wrap_y": n_y,
        "n_wrap_any": min(defined) if defined else -1,
        "occ_hash": occ_hash,
        "seq_hash": seq_hash,
        "seq": seq,
        "n_clusters_jam": len(cl),
        "n_nonwrapping_jam": sum(1 for c in cl if not (c[1] or c[2])),
        "owner": owner,
        "orient": orient,
        "snap_hist": snap_hist,
    }


def _fits(occ: np.ndarray, k: int, h_only: bool = False) -> np.ndarray:
    """Availability as a (2, L, L) boolean array: [o, y, x] is True when the
    placement (o, y, x) has k empty sites."""
    free = ~occ
    fits = np.ones((2,) + occ.shape, dtype=bool)
    for i in range(k):
        fits[0] &= np.roll(free, -i, axis=1)
        fits[1] &= np.roll(free, -i, axis=0)
    if h_only:
        fits[1] = False
    return fits


def changed_words(before: np.ndarray, after: np.ndarray) -> int:
    """Number of 64-bit availability words (orientation, row, column // 64)
    holding at least one placement whose availability differs."""
    diff = before != after
    L = diff.shape[2]
    W = (L + 63) // 64
    pad = np.zeros((2, L, W * 64), dtype=bool)
    pad[:, :, :L] = diff
    return int(pad.reshape(2, L, W, 64).any(axis=3).sum())


def word_changes(L: int, k: int, seed: int, sample: int, h_only: bool = False) -> dict:
    """Run the chain with availability recomputed from the occupancy after
    every deposit (no windings) and count, per step, the availability words
    whose value changes (Sec. II.B: each deposit makes every placement that
    covers one of its sites unviable).  Returns n_jam, the total changed-word
    count, and the number of availability bits that went from 1 to 0."""
    occ = np.zeros((L, L), dtype=bool)
    fits = _fits(occ, k, h_only)
    total_words = 0
    cleared = 0
    t = 0
    while True:
        av = np.flatnonzero(fits.ravel())
        A = len(av)
        if A == 0:
            break
        u = draw_u(seed, sample, t)
        P = int(av[(u * A) >> 64])
        o, rem = divmod(P, L * L)
        y, x = divmod(rem, L)
        for i in range(k):
            sy, sx = ((y + i) % L, x) if o else (y, (x + i) % L)
            occ[sy, sx] = True
        new = _fits(occ, k, h_only)
        assert not (new & ~fits).any()   # availability only ever drops
        total_words += changed_words(fits, new)
        cleared += int((fits & ~new).sum())
        fits = new
        t += 1
    return {"n_jam": t, "wchg_words": total_words, "bits_cleared": cleared}


def clusters_with_positions(occ: np.ndarray):
    """Clusters of occupied sites with breadth-first unwrapped coordinates:
    (label grid, {site: (ux, uy)}, [wraps per cluster]).  A cluster wraps when
    some edge disagrees with the offset of its two ends."""
    L = occ.shape[0]
    label = -np.ones((L, L), dtype=np.int64)
    pos = {}
    wraps = []
    for sy in range(L):
        for sx in range(L):
            if not occ[sy, sx] or label[sy, sx] >= 0:
                continue
            c = len(wraps)
            w = False
            label[sy, sx] = c
            pos[(sy, sx)] = (sx, sy)
            q = deque([(sy, sx)])
            while q:
                y, x = q.popleft()
                ux, uy = pos[(y, x)]
                for ex, ey in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    ny, nx = (y + ey) % L, (x + ex) % L
                    if not occ[ny, nx]:
                        continue
                    want = (ux + ex, uy + ey)
                    if label[ny, nx] < 0:
                        label[ny, nx] = c
                        pos[(ny, nx)] = want
                        q.append((ny, nx))
                    elif pos[(ny, nx)] != want:
                        w = True
            wraps.append(w)
    return label, pos, wraps


def paper_wrap_test(L: int, k: int, seed: int, sample: int) -> dict:
    """Run the chain and, at every deposit, apply the Sec. II.D test: for each
    pair of sites of one (not yet wrapping) cluster that the new k-mer touches,
    |x1 - x2| + |y1 - y2| over their unwrapped coordinates above 2k means a
    wrap.  Alongside, the exact winding of the cycle the pair closes through
    the new k-mer: (unwrapped offset of the two sites) minus (their offset
    along the new k-mer).  Returns the first step where the 2k test fires
    (1-based, -1 if never) and the number of pairs where the two disagree."""
    occ = np.zeros((L, L), dtype=bool)
    t = 0
    first = -1
    pairs = disagree = 0
    wrapped_before = False
    while True:
        fits = _fits(occ, k)
        av = np.flatnonzero(fits.ravel())
        A = len(av)
        if A == 0:
            break
        u = draw_u(seed, sample, t)
        P = int(av[(u * A) >> 64])
        o, rem = divmod(P, L * L)
        y, x = divmod(rem, L)
        label, pos, wraps = clusters_with_positions(occ)
        wrapped_before = wrapped_before or any(wraps)
        # contacts: (cluster, unwrapped site position, offset from the anchor
        # through the new k-mer)
        ux, uy = (1, 0) if o == 0 else (0, 1)
        touch = {}
        for i in range(k):
            ay, ax = (y + i * uy) % L, (x + i * ux) % L
            for ex, ey in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                by, bx = (ay + ey) % L, (ax + ex) % L
                if not occ[by, bx]:
                    continue
                c = int(label[by, bx])
                touch.setdefault(c, []).append((pos[(by, bx)], (i * ux + ex, i * uy + ey)))
        fired = False
        for c, lst in touch.items():
            if wraps[c]:
                continue
            for a in range(len(lst)):
                for b in range(a + 1, len(lst)):
                    (p1, r1), (p2, r2) = lst[a], lst[b]
                    manhattan = abs(p1[0] - p2[0]) + abs(p1[1] - p2[1])
                    wx = (p1[0] - p2[0]) - (r1[0] - r2[0])
                    wy = (p1[1] - p2[1]) - (r1[1] - r2[1])
                    paper = manhattan > 2 * k
                    pairs += 1
                    disagree += int(paper != (wx != 0 or wy != 0))
                    fired = fired or paper
        for i in range(k):
            occ[(y + i * uy) % L, (x + i * ux) % L] = True
        if fired and first < 0 and not wrapped_before:
            first = t + 1
        t += 1
    return {"n_jam": t, "first_2k": first, "pairs": pairs, "disagree": disagree}
