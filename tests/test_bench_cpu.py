"""bench.py's contract on the host: one GPU only, no CPU fallback for the
measured path, and the oracle leg (cpu_baseline) reports a bounded sample with
its parity against the results it is given."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    out = run_bench("--gpus", "2")
    assert out.returncode == 2
    assert "one GPU only" in out.stderr


def test_no_cpu_fallback_without_a_gpu():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = run_bench("--steps", "1", "--warmup", "0", "--serve-window", "0")
    assert out.returncode != 0
    assert "needs a GPU" in out.stderr
    assert not out.stdout.strip()   # no JSON line is printed


def test_cpu_baseline_sample_and_parity():
    import bench
    import oracle

    descs = [(16, 2, 5, s, 0) for s in range(12)] + [(24, 3, 6, s, 0) for s in range(12)]
    truth = oracle.run_many(descs)
    out = bench.cpu_baseline(descs, truth, budget_s=0.05)
    assert out["kind"] == "oracle" and out["unit"] == "deposits/s"
    assert 1 <= out["cores"] <= 16
    n = int(out["sample"].split()[1])
    assert 1 <= n <= len(descs) and out["parity"] == f"{n}/{n} bit-exact"
    assert out["value"] > 0
    # a wrong result in the sample is counted
    bad = [dict(r) for r in truth]
    bad[0]["occ_hash"] ^= 1
    out = bench.cpu_baseline(descs, bad, budget_s=0.05)
    n = int(out["sample"].split()[1])
    assert out["parity"] == f"{n - 1}/{n} bit-exact"
