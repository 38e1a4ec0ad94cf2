"""Writes large_expected.json: the oracle's results for every run of the two
large workloads (L = 16384, k = 1024, seed 4, samples 0..31 and L = 32768,
k = 4096, seed 5, samples 0..7), which the oracle takes minutes to compute.
Calls only the oracle; run from the repository root:

    python tests/golden/make_large_expected.py

The L = 32768 runs hold about 4.3 GiB each, so they go eight at a time.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

# (L, k, seed, sample, flags): every sample of both workloads
DESCS = [(16384, 1024, 4, s, 0) for s in range(32)] + [(32768, 4096, 5, s, 0) for s in range(8)]


def main():
    threads = max(1, min(8, os.cpu_count() or 1))
    t0 = time.time()
    res = oracle.run_many(DESCS, threads=threads)
    out = {"descs": DESCS, "results": res, "oracle_seconds": round(time.time() - t0, 1),
           "threads": threads}
    with open(os.path.join(HERE, "large_expected.json"), "w") as f:
        f.write("{\n")
        f.write(f' "descs": {json.dumps(DESCS)},\n')
        f.write(' "results": [\n')
        f.write(",\n".join("  " + json.dumps(r) for r in res))
        f.write("\n ],\n")
        f.write(f' "oracle_seconds": {out["oracle_seconds"]},\n "threads": {threads}\n}}\n')


if __name__ == "__main__":
    main()
