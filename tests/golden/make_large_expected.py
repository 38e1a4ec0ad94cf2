"""Writes large_expected.json: the oracle's results for sampled runs of the
two large workloads (L = 16384, k = 1024, seed 4 and L = 32768, k = 4096,
seed 5), which the oracle takes minutes each to compute.  Calls only the
oracle; run from the repository root:

    python tests/golden/make_large_expected.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

# (L, k, seed, sample, flags): samples 0, 17, 31 of the 32-sample workload
# and 0, 3, 7 of the 8-sample one
DESCS = [(16384, 1024, 4, s, 0) for s in (0, 17, 31)] + [(32768, 4096, 5, s, 0) for s in (0, 3, 7)]


def main():
    t0 = time.time()
    res = oracle.run_many(DESCS, threads=len(DESCS))
    out = {"descs": DESCS, "results": res, "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "large_expected.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
