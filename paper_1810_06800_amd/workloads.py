"""Seeded synthetic workloads: lists of (L, k, seed, sample, flags) descriptors.

This module holds none of the method's arithmetic; it only names the runs.
The paper's runs are single samples at L = 100k (Sec. II.A); the workloads
here are scaled to L/k = 8..64 and L <= 32768 so one MI355X can hold them.
Where a workload draws shapes at random it uses numpy's PCG64 generator,
which is unrelated to the Philox stream the method draws its placements from.
"""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

MIXED_SHAPES = [(256, 4), (512, 32), (1024, 64), (2048, 128), (4096, 256)]


def plain_small():
    """L = 64, k = 8, seed 1, samples 0..255."""
    return [(64, 8, 1, s, 0) for s in range(256)]


def plain_scale():
    """L = 1024, k = 64, seeds 0..1023, sample 0 each."""
    return [(1024, 64, j, 0, 0) for j in range(1024)]


def mixed_batch(n: int = 512, seed: int = 3):
    """n samples, seed 3, sample j; (L, k) uniform over MIXED_SHAPES."""
    rng = np.random.Generator(np.random.PCG64(seed))
    picks = rng.integers(0, len(MIXED_SHAPES), size=n)
    return [(MIXED_SHAPES[p][0], MIXED_SHAPES[p][1], seed, j, 0) for j, p in enumerate(picks.tolist())]


def large_16k():
    """L = 16384, k = 1024, seed 4, samples 0..31."""
    return [(16384, 1024, 4, s, 0) for s in range(32)]


def large_32k():
    """L = 32768, k = 4096, seed 5, samples 0..7."""
    return [(32768, 4096, 5, s, 0) for s in range(8)]


def serving_trace(requests: int = 1000, rate_hz: float = 200.0, seed: int = 2,
                  l_min: int = 256, l_max: int = 16384):
    """Poisson arrivals of jobs (L, k, n_samples): L a power of two in
    [l_min, l_max], k a power of two in [2, L/8], n uniform in [1, 64].
    Request r uses seed r and samples 0..n-1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = [1 << e for e in range(l_min.bit_length() - 1, l_max.bit_length())]
    t = 0.0
    out = []
    for r in range(requests):
        t += float(rng.exponential(1.0 / rate_hz))
        L = Ls[int(rng.integers(0, len(Ls)))]
        ks = [1 << e for e in range(1, (L // 8).bit_length())]
        k = ks[int(rng.integers(0, len(ks)))]
        n = int(rng.integers(1, 65))
        out.append({"id": r, "arrival_s": t, "L": L, "k": k, "n": n, "seed": r})
    return out


def save_trace(path: str, trace) -> None:
    with open(path, "w") as f:
        json.dump(trace, f)


def load_trace(path: str):
    with open(path) as f:
        return json.load(f)


CONFIGS = {
    "plain_small": plain_small,
    "plain_scale": plain_scale,
    "mixed_batch": mixed_batch,
    "large_16k": large_16k,
    "large_32k": large_32k,
}
