"""Serial CPU oracle for RSA of linear k-mers on an L x L torus (arXiv:1810.06800).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
imports it, and it imports nothing from the GPU library.

The C source (``rsa_oracle.c``) is the oracle; this module only builds it and
marshals arguments through ctypes.  Independent samples run on a thread pool
(ctypes releases the GIL during the call); each sample is serial.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rsa_oracle.c")
LIB = os.path.join(HERE, "librsa_oracle.so")

FLAG_H_ONLY = 1

STATUS_NAMES = {0: "ok", -1: "einval", -2: "enomem", -10: "escan", -11: "ecount",
                -12: "enowrap", -13: "eorder", -14: "ecapacity"}


class Desc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("k", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("sample", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("n_jam", ctypes.c_int64), ("n_wrap_x", ctypes.c_int64),
                ("n_wrap_y", ctypes.c_int64), ("n_wrap_any", ctypes.c_int64),
                ("occ_hash", ctypes.c_uint64), ("seq_hash", ctypes.c_uint64),
                ("n_clusters_jam", ctypes.c_int32), ("n_nonwrapping_jam", ctypes.c_int32),
                ("status", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("alg_bytes", ctypes.c_uint64), ("wchg_words", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "pad_"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``librsa_oracle.so``."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    """Load the oracle library, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.rsao_run.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Result),
                               ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint64, ctypes.c_int64,
                               ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64]
        L.rsao_run.restype = ctypes.c_int
        L.rsao_run_many.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Result), ctypes.c_uint32]
        L.rsao_run_many.restype = ctypes.c_int
        L.rsao_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(ctypes.c_uint32),
                                         ctypes.POINTER(ctypes.c_uint32)]
        L.rsao_philox4x32_10.restype = None
        L.rsao_mix64.argtypes = [ctypes.c_uint64]
        L.rsao_mix64.restype = ctypes.c_uint64
        L.rsao_rank.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.rsao_rank.restype = ctypes.c_uint32
        L.rsao_contacts_at_jamming.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_uint64)]
        L.rsao_contacts_at_jamming.restype = ctypes.c_int
        _lib = L
    return _lib


def _desc(L: int, k: int, seed: int, sample: int, flags: int = 0) -> Desc:
    return Desc(L, k, seed, sample, flags)


def philox(ctr, key):
    """Philox4x32-10 of a 4-word counter and a 2-word key."""
    c = (ctypes.c_uint32 * 4)(*ctr)
    kk = (ctypes.c_uint32 * 2)(*key)
    out = (ctypes.c_uint32 * 4)()
    lib().rsao_philox4x32_10(c, kk, out)
    return tuple(out)


def mix64(z: int) -> int:
    return lib().rsao_mix64(z)


def rank(u: int, a: int) -> int:
    return lib().rsao_rank(u, a)


def run(L: int, k: int, seed: int, sample: int, flags: int = 0, want_seq: bool = False,
        snap_step: int = 0, snap_cap: int = 0) -> dict:
    """Run one sample to jamming.  Returns the result fields as a dict, plus
    ``seq`` (list of canonical placement indices) and ``snap_hist`` on request."""
    d = _desc(L, k, seed, sample, flags)
    r = Result()
    cap = L * L // k + 1 if want_seq else 0
    seq = (ctypes.c_uint32 * cap)() if want_seq else None
    hist = (ctypes.c_uint64 * snap_cap)() if snap_cap else None
    lib().rsao_run(ctypes.byref(d), ctypes.byref(r), seq, cap, snap_step, hist, snap_cap)
    out = r.as_dict()
    if want_seq:
        out["seq"] = list(seq[: max(out["n_jam"], 0)])
    if snap_cap:
        out["snap_hist"] = list(hist)
    return out


def run_many(descs, threads: int | None = None) -> list[dict]:
    """Run many samples, one per thread at a time.  ``descs`` is a sequence of
    (L, k, seed, sample[, flags]) tuples; results come back in the same order."""
    descs = [tuple(d) + (0,) * (5 - len(d)) for d in descs]
    n = len(descs)
    if n == 0:
        return []
    threads = threads or os.cpu_count() or 1
    threads = max(1, min(threads, n))
    chunks = [list(range(i, n, threads)) for i in range(threads)]
    results: list[dict | None] = [None] * n
    library = lib()

    def work(idx):
        arr = (Desc * len(idx))(*[_desc(*descs[i]) for i in idx])
        res = (Result * len(idx))()
        library.rsao_run_many(arr, res, len(idx))
        for j, i in enumerate(idx):
            results[i] = res[j].as_dict()

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(work, chunks))
    return results  # type: ignore[return-value]


def contacts_at_jamming(L: int, k: int, seed: int, sample: int, flags: int = 0):
    """(n_x, n_y, n_xy) contact counts of the jammed state (Eq. 12)."""
    out = (ctypes.c_uint64 * 3)()
    d = _desc(L, k, seed, sample, flags)
    rc = lib().rsao_contacts_at_jamming(ctypes.byref(d), out)
    if rc != 0:
        raise RuntimeError(f"oracle status {rc}")
    return tuple(out)
