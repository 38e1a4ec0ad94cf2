"""ctypes binding of the C ABI in ``include/rsa.h`` (argument marshalling only).

Every step of the method runs in the HIP library; this module converts
descriptors and results, hands the library torch's current HIP stream and,
by default, torch's caching allocator for device memory.  It raises
``RuntimeError`` when the library is missing: there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Iterable, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsa_hip.so")
TILE_TABLE = os.path.join(HERE, "tiles.json")   # written by paper_1810_06800_amd.autotune

RSA_OK, RSA_EINVAL, RSA_ENOMEM, RSA_EDEVICE, RSA_ENOTREADY, RSA_EBUSY, RSA_ENOTFOUND = (
    0, -1, -2, -3, -4, -5, -6)
FLAG_H_ONLY = 1
FLAG_TRACK_CLUSTERS = 2
FLAG_CONTACTS = 4
FLAG_CLUSTER_SIZES = 8
SIZE_BINS = 32
OPT_MODE, OPT_TILE, OPT_GRAPH, OPT_SLOTS, OPT_PROFILE, OPT_IV_SLAB = 1, 2, 3, 4, 5, 6
PROFILE_SLOTS = ("init", "sel_total", "sel_ring", "sel_select", "sel_clear", "lab_total", "lab_idle",
                 "lab_map", "lab_gather", "lab_resolve", "lab_merge", "lab_writeback",
                 "lab_batches", "lab_edges", "lab_flushes", "steps", "spec_hits", "sel_hook",
                 "sel_process", "iv_cut", "iv_meet", "iv_rows")
MODE_BATCHED, MODE_PLAIN = 0, 1

# Symbols declared in include/rsa.h.
EXPORTS = ("rsa_create", "rsa_footprint_bytes", "rsa_run_batch", "rsa_results",
           "rsa_batch_elapsed_ms", "rsa_batch_profile", "rsa_batch_cluster_sizes", "rsa_destroy",
           "rsa_strerror", "rsa_last_error", "rsa_set_option", "rsa_get_option", "rsa_num_tiles",
           "rsa_tile_for_shape", "rsa_tile_shape", "rsa_set_tile_table", "rsa_tile_for_sample",
           "rsa_server_create", "rsa_server_submit", "rsa_server_step", "rsa_server_completed",
           "rsa_server_results", "rsa_server_stats", "rsa_server_destroy", "rsa_run_batch_static")
STATIC_SCRATCH_BYTES = 128 << 20   # RSA_STATIC_SCRATCH_BYTES
STATIC_MAX_SAMPLES = 2048          # RSA_STATIC_MAX_SAMPLES


class Sample(ctypes.Structure):
    _fields_ = [("L", ctypes.c_uint32), ("k", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("sample", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("n_jam", ctypes.c_int64), ("n_wrap_x", ctypes.c_int64),
                ("n_wrap_y", ctypes.c_int64), ("n_wrap_any", ctypes.c_int64),
                ("occ_hash", ctypes.c_uint64), ("seq_hash", ctypes.c_uint64),
                ("n_clusters_jam", ctypes.c_int32), ("n_nonwrapping_jam", ctypes.c_int32),
                ("status", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("alg_bytes", ctypes.c_uint64), ("wchg_words", ctypes.c_uint64),
                ("n_contacts_x", ctypes.c_int64), ("n_contacts_y", ctypes.c_int64),
                ("n_contacts_xy", ctypes.c_int64)]


RESULT_FIELDS = [name for name, _ in Result._fields_]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("quantum_us", ctypes.c_uint32),
                ("max_resident", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "requests_submitted", "requests_completed", "samples_queued", "samples_resident",
        "samples_completed", "deposits_completed", "deposits_in_progress", "arena_bytes",
        "arena_used", "arena_peak", "launches")]


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


class RsaError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        super().__init__(f"rsa error {code} ({strerror(code)}){': ' + msg if msg else ''}")


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``librsa_hip.so``; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1810_06800_amd.build` (hipcc, gfx950)")
    # torch ships its own HIP runtime: load it first so that the library
    # binds to the same one (loaded the other way round, two runtimes end up
    # in the process and the library sees no device)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.rsa_create.argtypes = [ctypes.POINTER(vp), i32, u64, ctypes.POINTER(Allocator)]
    L.rsa_create.restype = i32
    L.rsa_footprint_bytes.argtypes = [u32, u32]
    L.rsa_footprint_bytes.restype = ctypes.c_size_t
    L.rsa_run_batch.argtypes = [vp, ctypes.POINTER(Sample), u32, vp, ctypes.POINTER(u64)]
    L.rsa_run_batch.restype = i32
    L.rsa_run_batch_static.argtypes = [vp, ctypes.POINTER(Sample), u32, vp, vp]
    L.rsa_run_batch_static.restype = i32
    L.rsa_results.argtypes = [vp, u64, ctypes.POINTER(Result), u32, i32]
    L.rsa_results.restype = i32
    L.rsa_batch_elapsed_ms.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_float)]
    L.rsa_batch_elapsed_ms.restype = i32
    L.rsa_batch_profile.argtypes = [vp, u64, ctypes.POINTER(u64), u32, ctypes.POINTER(u32),
                                    ctypes.POINTER(u32)]
    L.rsa_batch_profile.restype = i32
    L.rsa_batch_cluster_sizes.argtypes = [vp, u64, ctypes.POINTER(u64), u32]
    L.rsa_batch_cluster_sizes.restype = i32
    L.rsa_destroy.argtypes = [vp]
    L.rsa_destroy.restype = None
    L.rsa_strerror.argtypes = [i32]
    L.rsa_strerror.restype = ctypes.c_char_p
    L.rsa_last_error.argtypes = [vp]
    L.rsa_last_error.restype = ctypes.c_char_p
    L.rsa_set_option.argtypes = [vp, i32, ctypes.c_int64]
    L.rsa_set_option.restype = i32
    L.rsa_get_option.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int64)]
    L.rsa_get_option.restype = i32
    L.rsa_num_tiles.argtypes = []
    L.rsa_num_tiles.restype = i32
    L.rsa_tile_for_shape.argtypes = [u32, u32]
    L.rsa_tile_for_shape.restype = i32
    ip = ctypes.POINTER(ctypes.c_int)
    L.rsa_tile_shape.argtypes = [i32, ip, ip, ip, ip]
    L.rsa_tile_shape.restype = i32
    L.rsa_set_tile_table.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                     ctypes.POINTER(ctypes.c_int32), u32]
    L.rsa_set_tile_table.restype = i32
    L.rsa_tile_for_sample.argtypes = [vp, u32, u32]
    L.rsa_tile_for_sample.restype = i32
    L.rsa_server_create.argtypes = [vp, ctypes.POINTER(ServerConfig), vp, ctypes.POINTER(vp)]
    L.rsa_server_create.restype = i32
    L.rsa_server_submit.argtypes = [vp, ctypes.POINTER(Sample), u32, ctypes.POINTER(u64)]
    L.rsa_server_submit.restype = i32
    L.rsa_server_step.argtypes = [vp, i32]
    L.rsa_server_step.restype = i32
    L.rsa_server_completed.argtypes = [vp, ctypes.POINTER(u64), u32]
    L.rsa_server_completed.restype = i32
    L.rsa_server_results.argtypes = [vp, u64, ctypes.POINTER(Result), u32]
    L.rsa_server_results.restype = i32
    L.rsa_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.rsa_server_stats.restype = i32
    L.rsa_server_destroy.argtypes = [vp]
    L.rsa_server_destroy.restype = None
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().rsa_strerror(code).decode()


def footprint_bytes(L: int, k: int) -> int:
    return lib().rsa_footprint_bytes(L, k)


def num_tiles() -> int:
    return lib().rsa_num_tiles()


def tile_for_shape(L: int, k: int) -> int:
    return lib().rsa_tile_for_shape(L, k)


def tile_shape(tile: int) -> tuple[int, int, int, int]:
    """(waves sharing select/clear, bitmap tile rows, map tile rows, sparse clear)."""
    a, b, c, d = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = lib().rsa_tile_shape(tile, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d))
    if rc != RSA_OK:
        raise RsaError(rc, "rsa_tile_shape")
    return a.value, b.value, c.value, d.value


def make_samples(descs: Iterable[Sequence[int]]):
    """(L, k, seed, sample[, flags]) tuples -> a ctypes array of rsa_sample_t."""
    descs = [tuple(int(v) for v in d) for d in descs]
    arr = (Sample * max(len(descs), 1))()
    for i, d in enumerate(descs):
        L, k, seed, sample = d[:4]
        flags = d[4] if len(d) > 4 else 0
        arr[i] = Sample(L, k, seed & (2**64 - 1), sample, flags)
    return arr, len(descs)


def _torch_allocator(device: int):
    """rsa_allocator_t backed by torch's caching allocator on `device`."""
    import torch

    def alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except Exception:  # out of memory: the library reports RSA_ENOMEM
            return None

    def free(ptr, _nbytes, _user):
        # a context finalised while the interpreter shuts down may outlive
        # torch's module state; its memory goes back with the process then
        cuda = getattr(torch, "cuda", None)
        delete = getattr(cuda, "caching_allocator_delete", None) if cuda is not None else None
        if delete is None:
            return
        try:
            delete(ptr)
        except Exception:
            pass

    fa, ff = ALLOC_FN(alloc), FREE_FN(free)
    return Allocator(fa, ff, None), (fa, ff)


def load_tile_table(path: str = TILE_TABLE):
    """[(L, k, tile)] from an autotune table file ([] if it does not exist)."""
    import json

    if not path or not os.path.exists(path):
        return []
    with open(path) as f:
        t = json.load(f)
    return [(int(e["L"]), int(e["k"]), int(e["tile"])) for e in t["entries"]]


_live_contexts: "weakref.WeakSet" = None


def _close_live_contexts():
    """atexit hook: destroy contexts still open, while torch is intact."""
    for ctx in list(_live_contexts or ()):
        try:
            ctx.close()
        except Exception:
            pass


class Context:
    """An rsa_ctx on one device.  ``allocator='torch'`` (default) takes device
    memory from torch's caching allocator; ``'hip'`` lets the library call
    hipMalloc.  Work goes to torch's current stream unless a stream is given.
    ``tile_table`` is the autotune table file handed to the library (the
    package's tiles.json by default; None for the built-in heuristic only)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, allocator: str = "torch",
                 tile_table: str | None = TILE_TABLE):
        self._lib = lib()
        self.device = device
        self._keep = None
        alloc_ptr = None
        if allocator == "torch":
            import torch

            torch.cuda.init()
            alloc, self._keep = _torch_allocator(device)
            self._alloc = alloc
            alloc_ptr = ctypes.byref(alloc)
        elif allocator != "hip":
            raise ValueError("allocator must be 'torch' or 'hip'")
        handle = ctypes.c_void_p()
        rc = self._lib.rsa_create(ctypes.byref(handle), device, budget_bytes, alloc_ptr)
        if rc != RSA_OK:
            raise RsaError(rc, "rsa_create")
        self._h = handle
        global _live_contexts
        if _live_contexts is None:
            _live_contexts = weakref.WeakSet()
            atexit.register(_close_live_contexts)
        _live_contexts.add(self)
        self.set_tile_table(load_tile_table(tile_table) if tile_table else [])

    def set_tile_table(self, entries) -> None:
        """Hand the library an autotune table: [(L, k, tile)]."""
        n = len(entries)
        Ls = (ctypes.c_uint32 * max(n, 1))(*[e[0] for e in entries])
        ks = (ctypes.c_uint32 * max(n, 1))(*[e[1] for e in entries])
        ts = (ctypes.c_int32 * max(n, 1))(*[e[2] for e in entries])
        rc = self._lib.rsa_set_tile_table(self._h, Ls, ks, ts, n)
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())

    def tile_for_sample(self, L: int, k: int) -> int:
        rc = self._lib.rsa_tile_for_sample(self._h, L, k)
        if rc < 0:
            raise RsaError(rc, self.last_error())
        return rc

    # -- options
    def set_option(self, option: int, value: int) -> None:
        rc = self._lib.rsa_set_option(self._h, option, value)
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        rc = self._lib.rsa_get_option(self._h, option, ctypes.byref(v))
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        return v.value

    def last_error(self) -> str:
        return self._lib.rsa_last_error(self._h).decode()

    # -- batches
    def run_batch(self, descs, stream=None) -> tuple[int, int]:
        """Enqueue samples; returns (batch_id, n)."""
        arr, n = make_samples(descs)
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(self.device).cuda_stream
        bid = ctypes.c_uint64()
        rc = self._lib.rsa_run_batch(self._h, arr, n, ctypes.c_void_p(stream), ctypes.byref(bid))
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        return bid.value, n

    def run_batch_static(self, descs, out=None, stream=None):
        """rsa_run_batch_static: enqueue samples with no allocation inside the
        library; results go to ``out``, a device tensor of at least
        n * sizeof(rsa_result_t) bytes (a fresh uint8 tensor from torch when
        None).  Returns ``out``; read it with ``static_results`` after the
        stream has reached it."""
        import torch

        arr, n = make_samples(descs)
        nbytes = n * ctypes.sizeof(Result)
        if out is None:
            out = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        if not out.is_cuda or out.numel() * out.element_size() < nbytes or not out.is_contiguous():
            raise ValueError("out must be a contiguous device tensor of n * sizeof(rsa_result_t) bytes")
        if stream is None:
            stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = self._lib.rsa_run_batch_static(self._h, arr, n, ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(stream))
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        return out

    @staticmethod
    def static_results(out, n: int) -> list[dict]:
        """Results written by run_batch_static into ``out`` (copied to the host
        on the current stream)."""
        raw = out.view(-1)[: n * ctypes.sizeof(Result)].cpu().numpy().tobytes()
        arr = (Result * max(n, 1)).from_buffer_copy(raw.ljust(max(n, 1) * ctypes.sizeof(Result), b"\0"))
        return [{f: getattr(arr[i], f) for f in RESULT_FIELDS} for i in range(n)]

    def elapsed_ms(self, batch) -> float:
        bid = batch[0] if isinstance(batch, tuple) else batch
        ms = ctypes.c_float()
        rc = self._lib.rsa_batch_elapsed_ms(self._h, bid, ctypes.byref(ms))
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        return float(ms.value)

    def profile(self, batch):
        """Per-sample phase counters of a batch run with OPT_PROFILE = 1:
        (list of dicts, tick rate in kHz)."""
        bid, n = batch
        slots, khz = ctypes.c_uint32(), ctypes.c_uint32()
        out = (ctypes.c_uint64 * (max(n, 1) * len(PROFILE_SLOTS)))()
        rc = self._lib.rsa_batch_profile(self._h, bid, out, n, ctypes.byref(slots), ctypes.byref(khz))
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        m = slots.value
        assert m == len(PROFILE_SLOTS)
        return [dict(zip(PROFILE_SLOTS, out[i * m:(i + 1) * m])) for i in range(n)], khz.value

    def cluster_sizes(self, batch):
        """Cluster-size histograms of a batch (RSA_FLAG_CLUSTER_SIZES): one
        list of SIZE_BINS counts per sample, bin b = clusters of 2^b .. 2^(b+1)-1
        sites right after deposit n_wrap_any.  Call before results()."""
        bid, n = batch
        out = (ctypes.c_uint64 * (max(n, 1) * SIZE_BINS))()
        rc = self._lib.rsa_batch_cluster_sizes(self._h, bid, out, n)
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        return [list(out[i * SIZE_BINS:(i + 1) * SIZE_BINS]) for i in range(n)]

    def results(self, batch, wait: bool = True, as_array: bool = False):
        """Results of a batch as a list of dicts, or with as_array=True as a
        numpy structured array with the fields of rsa_result_t (None if not
        ready and wait=False)."""
        bid, n = batch
        out = (Result * max(n, 1))()
        rc = self._lib.rsa_results(self._h, bid, out, n, 1 if wait else 0)
        if rc == RSA_ENOTREADY:
            return None
        if rc != RSA_OK:
            raise RsaError(rc, self.last_error())
        if as_array:
            return np.ctypeslib.as_array(out)[:n].copy()
        return [{f: getattr(out[i], f) for f in RESULT_FIELDS} for i in range(n)]

    def run(self, descs, stream=None):
        return self.results(self.run_batch(descs, stream))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.rsa_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """An rsa_server on a Context: requests of (L, k, seed, sample[, flags])
    descriptors are queued by ``submit``, admitted by footprint and run in
    time-sliced launches by ``step``; ``completed`` and ``results`` collect
    them."""

    def __init__(self, ctx: Context, arena_bytes: int = 0, quantum_us: int = 0,
                 max_resident: int = 0, stream=None):
        self._lib = ctx._lib
        self.ctx = ctx
        if stream is None:
            import torch

            stream = torch.cuda.current_stream(ctx.device).cuda_stream
        cfg = ServerConfig(arena_bytes, quantum_us, max_resident)
        h = ctypes.c_void_p()
        rc = self._lib.rsa_server_create(ctx._h, ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(h))
        if rc != RSA_OK:
            raise RsaError(rc, ctx.last_error())
        self._h = h
        self._sizes = {}

    def submit(self, descs) -> int:
        arr, n = make_samples(descs)
        rid = ctypes.c_uint64()
        rc = self._lib.rsa_server_submit(self._h, arr, n, ctypes.byref(rid))
        if rc != RSA_OK:
            raise RsaError(rc, self.ctx.last_error())
        self._sizes[rid.value] = n
        return rid.value

    def step(self, wait: bool = False) -> int:
        rc = self._lib.rsa_server_step(self._h, 1 if wait else 0)
        if rc < 0:
            raise RsaError(rc, self.ctx.last_error())
        return rc

    def completed(self, cap: int = 4096) -> list[int]:
        ids = (ctypes.c_uint64 * cap)()
        n = self._lib.rsa_server_completed(self._h, ids, cap)
        if n < 0:
            raise RsaError(n, self.ctx.last_error())
        return [ids[i] for i in range(n)]

    def results(self, request_id: int):
        """Results of a completed request (list of dicts), or None if it has
        not completed yet."""
        n = self._sizes[request_id]
        out = (Result * n)()
        rc = self._lib.rsa_server_results(self._h, request_id, out, n)
        if rc == RSA_ENOTREADY:
            return None
        if rc != RSA_OK:
            raise RsaError(rc, self.ctx.last_error())
        del self._sizes[request_id]
        return [{f: getattr(out[i], f) for f in RESULT_FIELDS} for i in range(n)]

    def stats(self) -> dict:
        st = ServerStats()
        rc = self._lib.rsa_server_stats(self._h, ctypes.byref(st))
        if rc != RSA_OK:
            raise RsaError(rc, self.ctx.last_error())
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def run(self, requests, max_steps: int = 1 << 20) -> list[list[dict]]:
        """Submit every request at once and step until all have completed
        (RuntimeError after max_steps rounds)."""
        ids = [self.submit(r) for r in requests]
        done = {}
        for _ in range(max_steps):
            if len(done) == len(ids):
                break
            self.step(wait=True)
            for rid in self.completed():
                done[rid] = self.results(rid)
        else:
            raise RuntimeError(f"{len(ids) - len(done)} requests unfinished after {max_steps} steps")
        return [done[i] for i in ids]

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.rsa_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def results_array(results: list[dict]) -> np.ndarray:
    """Results as a numpy structured array (for vectorised checks)."""
    dt = np.dtype([(f, np.int64 if f not in ("occ_hash", "seq_hash", "alg_bytes", "wchg_words")
                    else np.uint64) for f in RESULT_FIELDS])
    return np.array([tuple(r[f] for f in RESULT_FIELDS) for r in results], dtype=dt)
