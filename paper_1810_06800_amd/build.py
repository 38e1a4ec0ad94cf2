"""Build the gfx950 library (HIP kernels + C ABI) in-tree with hipcc.

The kernel source is compiled once per wave-count index (each unit holds the
four persistent-kernel instantiations of one wave count), all units in
parallel, and linked with the host runtime into ``librsa_hip.so``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librsa_hip.so")
KERNEL_SOURCE = "rsa_kernels.hip"
NUM_WAVE_TILES = 5
HOST_SOURCES = ["rsa_capi.hip", "rsa_server.hip"]
ARCH = os.environ.get("RSA_OFFLOAD_ARCH", "gfx950")

# Every HIP translation unit is compiled without packed FP32 instructions.
HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-result"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build the library")
    return exe


def _run(cmd):
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + proc.stderr[-4000:])
    return proc.stderr


def units():
    """(source, object, extra flags) of every translation unit."""
    out = []
    for w in range(NUM_WAVE_TILES):
        out.append((KERNEL_SOURCE, f"rsa_kernels_w{w}.o", [f"-DRSA_TU_WAVES={w}"]))
    for src in HOST_SOURCES:
        out.append((src, src.replace(".hip", ".o"), []))
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile ``librsa_hip.so`` (always recompiles)."""
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    cmds = [[cc, *HIPCC_FLAGS, *extra, "-c", "-o", os.path.join(OBJ, obj), os.path.join(CSRC, src)]
            for src, obj, extra in units()]
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1))
    with ThreadPoolExecutor(jobs) as ex:
        logs = list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    logs.append(_run([cc, *HIPCC_FLAGS, "-shared", "-o", tmp,
                      *[os.path.join(OBJ, obj) for _, obj, _ in units()]]))
    if verbose:
        for log in logs:
            if log:
                print(log)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
