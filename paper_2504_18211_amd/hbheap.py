"""Thin ctypes binding of the C ABI in ``include/hbheap.h``.

Argument marshalling only: every step of allocation, free, trim and the
payload check runs in the HIP kernels of ``libhbheap.so``.  torch provides
device buffers (tensors on ``cuda``) and streams; functions take tensors or
raw device addresses (ints).  The library must be built first
(``__graft_entry__.build()``); loading fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhbheap.so")
# the test build with schedule fuzzing (the allocator only: no growth,
# serving or plain-baseline entry points); see use_fuzz_library()
FUZZ_LIB_PATH = os.path.join(HERE, "libhbheap_fuzz.so")

VARIANT_CHUNK, VARIANT_PAGE, VARIANT_VA_PAGE, VARIANT_VA_CHUNK, VARIANT_VL_PAGE, VARIANT_VL_CHUNK = 0, 1, 2, 3, 4, 5
OK, E_INVAL, E_NOMEM, E_HIP, E_RANGE, E_UNSUP = 0, -1, -2, -3, -4, -5
ERR_DOUBLE_FREE, ERR_INVALID_FREE, ERR_TIMEOUT, ERR_CORRUPT = 0x1, 0x2, 0x4, 0x8
FLAG_STATS, FLAG_VERIFY, FLAG_HOME0, FLAG_EAGER = 0x1, 0x2, 0x4, 0x8
STAT_NAMES = ["chunk_grabs", "refills", "oom", "oom_waits", "double_free", "invalid_free", "timeouts", "reserved7",
              "state_ops", "headtail_ops", "pool_ops", "spread_ops", "retired", "slot_ops", "reserved14",
              "reserved15"]
FREE_OK, FREE_DOUBLE, FREE_INVALID, FREE_NULL = 0, 1, 2, 3

EXPORTS = [
    "heap_create", "heap_create_ex", "heap_destroy", "heap_alloc_batch", "heap_free_batch", "heap_free_batch_ex",
    "heap_device_handle", "heap_set_flags", "heap_info", "heap_trim", "heap_snapshot", "heap_get_error", "heap_clear_error",
    "heap_stats", "heap_replay", "heap_pattern_write", "heap_pattern_check", "hb_atomic_probe", "hb_stream_copy",
    "hb_plain_set_heap", "hb_plain_alloc", "hb_plain_free", "hb_plain_pattern", "hbheap_version",
    "growth_create", "growth_destroy", "growth_step", "growth_graph_launch", "growth_release", "growth_export",
    "growth_launch_shape", "growth_autotune",
    "serve_create", "serve_destroy", "serve_run", "serve_export", "heap_chunks_in_use",
    "heap_chunks_in_use_noalloc", "hb_fuzz_set", "hb_host_malloc_sweep",
]
SERVE_OK, SERVE_FREE_DOUBLE, SERVE_FREE_INVAL, SERVE_FREE_NULL, SERVE_ALLOC_NULL = 0, 1, 2, 3, 4


class HbHeapError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} returned {code}")
        self.code = code


class HeapConfig(C.Structure):
    _fields_ = [("variant", C.c_uint32), ("width", C.c_uint32), ("spin_cap", C.c_uint32),
                ("backoff_max", C.c_uint32), ("flags", C.c_uint32), ("shards", C.c_uint32), ("rows", C.c_uint32)]


class HeapInfo(C.Structure):
    _fields_ = [("data", C.c_void_p), ("data_bytes", C.c_uint64), ("chunk_bytes", C.c_uint64),
                ("n_chunks", C.c_uint64), ("n_classes", C.c_uint32), ("variant", C.c_uint32),
                ("ring_entries", C.c_uint64), ("state_bytes", C.c_uint64), ("metadata_bytes", C.c_uint64),
                ("n_shards", C.c_uint32), ("reserved", C.c_uint32)]


class GrowthCandidate(C.Structure):
    _fields_ = [("chunk_bytes", C.c_uint64), ("variant", C.c_uint32), ("width", C.c_uint32), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]


class ServeConfig(C.Structure):
    _fields_ = [("slots", C.c_uint32), ("max_batch", C.c_uint32), ("max_requests", C.c_uint64),
                ("admit", C.c_double), ("seed", C.c_uint32), ("free_lag", C.c_uint32)]


class ServeStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("batches", "requests", "allocs", "frees", "trims", "admission_stalls",
                                          "monitor_reads", "peak_bound", "final_chunks")] + [("wall_s", C.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class DevHandle(C.Structure):
    """Mirror of hbheap_dev_t (passed by value to user kernels)."""
    _fields_ = [(n, C.c_void_p) for n in ("data", "state", "pool", "classes", "chunk_class", "chunk_cnt", "bits",
                                          "pool_ids", "slots", "err", "stats")] + \
               [("data_bytes", C.c_uint64)] + \
               [(n, C.c_uint32) for n in ("n_chunks", "log2_chunk", "n_classes", "variant", "words_per_chunk",
                                          "log2q", "width", "spin_cap", "backoff_max", "flags", "n_shards",
                                          "log2_span")] + \
               [(n, C.c_void_p) for n in ("vdir", "vtaken", "vstore", "vstore_slots")] + \
               [(n, C.c_uint32) for n in ("log2_seg", "log2_dir", "log2_store", "vsegs")] + \
               [("vbudget", C.c_uint64), ("chunk_ct", C.c_void_p)]


_lib = None
_libs = {}
_path = LIB_PATH


def use_fuzz_library(on: bool):
    """Route every later call through the schedule-fuzzing test build (on)
    or the normal library (off).  Heaps must be used with the library that
    created them."""
    global _lib, _path
    _path = FUZZ_LIB_PATH if on else LIB_PATH
    _lib = _libs.get(_path)


def lib():
    """Load libhbheap.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_path):
        raise RuntimeError(f"{_path} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no fallback")
    L = C.CDLL(_path)
    vp, sz, u32, i32, i64p = C.c_void_p, C.c_size_t, C.c_uint32, C.c_int, C.c_void_p
    sig = {
        "heap_create": [sz, sz, C.POINTER(vp)],
        "heap_create_ex": [sz, sz, C.POINTER(HeapConfig), C.POINTER(vp)],
        "heap_destroy": [vp],
        "heap_alloc_batch": [vp, vp, vp, sz, vp],
        "heap_free_batch": [vp, vp, vp, sz, vp],
        "heap_free_batch_ex": [vp, vp, vp, sz, vp, vp],
        "heap_device_handle": [vp, C.POINTER(DevHandle)],
        "heap_set_flags": [vp, u32],
        "heap_info": [vp, C.POINTER(HeapInfo)],
        "heap_trim": [vp, vp],
        "heap_snapshot": [vp, vp, sz, C.POINTER(sz), vp],
        "heap_get_error": [vp, C.POINTER(u32)],
        "heap_clear_error": [vp],
        "heap_stats": [vp, C.POINTER(C.c_uint64)],
        "heap_replay": [vp, i64p, i64p, sz, vp],
        "heap_pattern_write": [vp, vp, vp, sz, u32, vp],
        "heap_pattern_check": [vp, vp, vp, sz, u32, vp, vp],
        "hb_atomic_probe": [i32, vp, sz, sz, u32, u32, vp],
        "hb_stream_copy": [vp, vp, sz, vp],
        "hb_plain_set_heap": [sz],
        "hb_plain_alloc": [vp, vp, sz, vp],
        "hb_plain_free": [vp, sz, vp],
        "hb_plain_pattern": [vp, vp, sz, u32, vp, vp],
        "growth_create": [vp, u32, vp, u32, u32, C.POINTER(vp)],
        "growth_destroy": [vp],
        "growth_step": [vp, u32, vp],
        "growth_graph_launch": [vp, vp],
        "growth_release": [vp, vp],
        "growth_export": [vp, vp, vp, vp, vp],
        "growth_launch_shape": [vp, C.POINTER(u32), C.POINTER(u32)],
        "growth_autotune": [sz, u32, vp, u32, u32, C.POINTER(GrowthCandidate), u32, u32, C.POINTER(C.c_float),
                            C.POINTER(C.c_int32)],
        "serve_create": [vp, C.POINTER(ServeConfig), C.POINTER(vp)],
        "serve_destroy": [vp],
        "serve_run": [vp, u32, vp, vp, vp, i32, vp, vp, vp, vp, vp, C.POINTER(ServeStats)],
        "serve_export": [vp, C.c_uint64, C.c_uint64, vp, vp],
        "heap_chunks_in_use": [vp, C.POINTER(C.c_uint64), vp],
        "heap_chunks_in_use_noalloc": [vp, vp, vp],
        "hb_fuzz_set": [u32, u32],
        "hb_host_malloc_sweep": [vp, u32, C.c_uint64, u32, u32, vp, C.POINTER(C.c_uint64)],
    }
    for name, args in sig.items():
        if _path == FUZZ_LIB_PATH and not hasattr(L, name):
            continue  # an entry point of another translation unit
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = args
    L.hbheap_version.restype = C.c_char_p
    L.hbheap_version.argtypes = []
    _lib = L
    _libs[_path] = L
    return L


def hb_host_malloc_sweep(sizes, requests: int, iterations: int, threads: int):
    """Host malloc/free rounds (no GPU): returns (seconds[n_sizes, iterations], failed)."""
    import numpy as np
    sz = np.ascontiguousarray(sizes, dtype=np.uint64)
    secs = np.zeros((len(sz), iterations), dtype=np.float64)
    failed = C.c_uint64()
    _check("hb_host_malloc_sweep", lib().hb_host_malloc_sweep(sz.ctypes.data, len(sz), requests, iterations, threads,
                                                              secs.ctypes.data, C.byref(failed)))
    return secs, int(failed.value)


def hb_fuzz_set(seed: int, most_sleeps: int = 32):
    _check("hb_fuzz_set", lib().hb_fuzz_set(seed, most_sleeps))


def _check(fn: str, rc: int):
    if rc != OK:
        raise HbHeapError(fn, rc)


def _addr(x) -> int | None:
    """Device address of a tensor (must live on the GPU) or an int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_cuda:
        raise ValueError("device buffer expected (a CUDA tensor)")
    return x.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# C ABI, same names
# ---------------------------------------------------------------------------

def heap_create(nbytes: int, chunk_bytes: int, variant: int = VARIANT_CHUNK, width: int = 64,
                spin_cap: int = 0, backoff_max: int = 0, flags: int = 0, shards: int = 0, rows: int = 0) -> int:
    cfg = HeapConfig(variant, width, spin_cap, backoff_max, flags, shards, rows)
    out = C.c_void_p()
    _check("heap_create_ex", lib().heap_create_ex(nbytes, chunk_bytes, C.byref(cfg), C.byref(out)))
    return out.value


def heap_destroy(h: int):
    _check("heap_destroy", lib().heap_destroy(h))


def heap_alloc_batch(h: int, sizes, ptrs, n: int | None = None, stream=None):
    n = sizes.numel() if n is None else n
    _check("heap_alloc_batch", lib().heap_alloc_batch(h, _addr(sizes), _addr(ptrs), n, _stream(stream)))


def heap_free_batch(h: int, sizes, ptrs, n: int | None = None, stream=None, status=None):
    n = ptrs.numel() if n is None else n
    _check("heap_free_batch_ex",
           lib().heap_free_batch_ex(h, _addr(sizes), _addr(ptrs), n, _addr(status), _stream(stream)))


def heap_set_flags(h: int, flags: int):
    _check("heap_set_flags", lib().heap_set_flags(h, flags))


def heap_device_handle(h: int) -> DevHandle:
    d = DevHandle()
    _check("heap_device_handle", lib().heap_device_handle(h, C.byref(d)))
    return d


def heap_info(h: int) -> HeapInfo:
    i = HeapInfo()
    _check("heap_info", lib().heap_info(h, C.byref(i)))
    return i


def heap_trim(h: int, stream=None):
    _check("heap_trim", lib().heap_trim(h, _stream(stream)))


def heap_snapshot(h: int, stream=None) -> bytes:
    n = C.c_size_t()
    _check("heap_snapshot", lib().heap_snapshot(h, None, 0, C.byref(n), _stream(stream)))
    buf = (C.c_uint8 * n.value)()
    _check("heap_snapshot", lib().heap_snapshot(h, buf, n.value, C.byref(n), _stream(stream)))
    return bytes(buf)


def heap_get_error(h: int) -> int:
    e = C.c_uint32()
    _check("heap_get_error", lib().heap_get_error(h, C.byref(e)))
    return e.value


def heap_clear_error(h: int):
    _check("heap_clear_error", lib().heap_clear_error(h))


def heap_stats(h: int) -> dict:
    a = (C.c_uint64 * len(STAT_NAMES))()  # heap_stats_t: one u64 field per counter, in order
    _check("heap_stats", lib().heap_stats(h, a))
    return {name: int(a[i]) for i, name in enumerate(STAT_NAMES)}


def heap_replay(h: int, ops, out, n: int | None = None, stream=None):
    n = ops.numel() if n is None else n
    _check("heap_replay", lib().heap_replay(h, _addr(ops), _addr(out), n, _stream(stream)))


def heap_pattern_write(h: int, ptrs, sizes, seed: int, n: int | None = None, stream=None):
    n = ptrs.numel() if n is None else n
    _check("heap_pattern_write", lib().heap_pattern_write(h, _addr(ptrs), _addr(sizes), n, seed & 0xFFFFFFFF,
                                                          _stream(stream)))


def heap_pattern_check(h: int, ptrs, sizes, seed: int, mismatches, n: int | None = None, stream=None):
    n = ptrs.numel() if n is None else n
    _check("heap_pattern_check", lib().heap_pattern_check(h, _addr(ptrs), _addr(sizes), n, seed & 0xFFFFFFFF,
                                                          _addr(mismatches), _stream(stream)))


def hb_atomic_probe(pattern: int, buf, buf_bytes: int, threads: int, lines: int, iters: int, stream=None):
    _check("hb_atomic_probe", lib().hb_atomic_probe(pattern, _addr(buf), buf_bytes, threads, lines, iters,
                                                    _stream(stream)))


def hb_stream_copy(dst, src, nbytes: int, stream=None):
    _check("hb_stream_copy", lib().hb_stream_copy(_addr(dst), _addr(src), nbytes, _stream(stream)))


def hb_plain_set_heap(nbytes: int) -> int:
    return lib().hb_plain_set_heap(nbytes)


def hb_plain_alloc(sizes, ptrs, n: int | None = None, stream=None):
    n = sizes.numel() if n is None else n
    _check("hb_plain_alloc", lib().hb_plain_alloc(_addr(sizes), _addr(ptrs), n, _stream(stream)))


def hb_plain_free(ptrs, n: int | None = None, stream=None):
    n = ptrs.numel() if n is None else n
    _check("hb_plain_free", lib().hb_plain_free(_addr(ptrs), n, _stream(stream)))


def hb_plain_pattern(ptrs, sizes, seed: int, mismatches=None, n: int | None = None, stream=None):
    """Write (mismatches None) or check the payload words in blocks of the
    runtime's allocator."""
    n = ptrs.numel() if n is None else n
    _check("hb_plain_pattern", lib().hb_plain_pattern(_addr(ptrs), _addr(sizes), n, seed, _addr(mismatches),
                                                      _stream(stream)))


def hbheap_version() -> str:
    return lib().hbheap_version().decode()


# ---- serving line (include/hbheap_serve.h) ----

def serve_create(h: int, slots: int, max_batch: int, max_requests: int, admit: float, seed: int,
                 free_lag: int) -> int:
    cfg = ServeConfig(slots, max_batch, max_requests, admit, seed & 0xFFFFFFFF, free_lag)
    out = C.c_void_p()
    _check("serve_create", lib().serve_create(h, C.byref(cfg), C.byref(out)))
    return out.value


def serve_destroy(s: int):
    _check("serve_destroy", lib().serve_destroy(s))


def _host(a, dtype):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def serve_run(s: int, first, ops, arrival_ns=None, alone: bool = False):
    """Host arrays in (numpy); returns dict of per-request status, cls, sum
    and per-batch latency_ns, wait_ns, plus the run's stats."""
    import numpy as np
    nb = len(first) - 1
    first, pf = _host(first, np.uint64)
    ops, po = _host(ops, np.int64)
    if arrival_ns is not None:
        arrival_ns, pa = _host(arrival_ns, np.uint64)
    else:
        pa = None
    R = int(first[-1]) if nb else 0
    status = np.zeros(R, dtype=np.uint8)
    cls = np.zeros(R, dtype=np.int8)
    sums = np.zeros(R, dtype=np.uint32)
    lat = np.zeros(nb, dtype=np.uint64)
    wait = np.zeros(nb, dtype=np.uint64)
    st = ServeStats()
    _check("serve_run", lib().serve_run(s, nb, pf, po, pa, 1 if alone else 0, status.ctypes.data, cls.ctypes.data,
                                        sums.ctypes.data, lat.ctypes.data, wait.ctypes.data, C.byref(st)))
    return {"status": status, "cls": cls, "sum": sums, "latency_ns": lat, "wait_ns": wait, "stats": st.as_dict()}


def serve_export(s: int, first: int, n: int, dst, stream=None):
    _check("serve_export", lib().serve_export(s, first, n, _addr(dst), _stream(stream)))


def heap_chunks_in_use(h: int, stream=None) -> int:
    v = C.c_uint64()
    _check("heap_chunks_in_use", lib().heap_chunks_in_use(h, C.byref(v), _stream(stream)))
    return v.value


def heap_chunks_in_use_noalloc(h: int, out, stream=None):
    """out: a device tensor of one int64, written in stream order."""
    _check("heap_chunks_in_use_noalloc", lib().heap_chunks_in_use_noalloc(h, _addr(out), _stream(stream)))



# ---- growth line (include/hbheap_growth.h) ----

def growth_create(h: int, agents: int, doublings, steps: int, seed: int) -> int:
    out = C.c_void_p()
    _check("growth_create", lib().growth_create(h, agents, _addr(doublings), steps, seed & 0xFFFFFFFF, C.byref(out)))
    return out.value


def growth_destroy(g: int):
    _check("growth_destroy", lib().growth_destroy(g))


def growth_step(g: int, step: int, stream=None):
    _check("growth_step", lib().growth_step(g, step, _stream(stream)))


def growth_graph_launch(g: int, stream=None):
    _check("growth_graph_launch", lib().growth_graph_launch(g, _stream(stream)))


def growth_release(g: int, stream=None):
    _check("growth_release", lib().growth_release(g, _stream(stream)))


def growth_export(g: int, ptrs=None, nbytes=None, failures=None, stream=None):
    _check("growth_export", lib().growth_export(g, _addr(ptrs), _addr(nbytes), _addr(failures), _stream(stream)))


def growth_launch_shape(g: int) -> tuple[int, int]:
    b, t = C.c_uint32(), C.c_uint32()
    _check("growth_launch_shape", lib().growth_launch_shape(g, C.byref(b), C.byref(t)))
    return b.value, t.value


def growth_autotune(heap_bytes: int, agents: int, doublings, steps: int, seed: int, candidates, reps: int):
    """candidates: list of (chunk_bytes, variant, width[, flags]).  Returns
    (median ms per candidate, negative where it could not run; index of the
    best)."""
    n = len(candidates)
    arr = (GrowthCandidate * n)(*[GrowthCandidate(*(tuple(c) + (0,))[:4], 0) for c in candidates])
    ms = (C.c_float * n)()
    best = C.c_int32()
    _check("growth_autotune", lib().growth_autotune(heap_bytes, agents, _addr(doublings), steps, seed & 0xFFFFFFFF,
                                                    arr, n, reps, ms, C.byref(best)))
    return [float(x) for x in ms], best.value


# ---------------------------------------------------------------------------
# convenience owner of a heap handle
# ---------------------------------------------------------------------------

class Heap:
    """Owns one heap; methods forward to the C ABI above."""

    def __init__(self, nbytes: int, chunk_bytes: int = 8192, variant: int = VARIANT_CHUNK, width: int = 64,
                 spin_cap: int = 0, backoff_max: int = 0, flags: int = 0, shards: int = 0, rows: int = 0):
        self.h = heap_create(nbytes, chunk_bytes, variant, width, spin_cap, backoff_max, flags, shards, rows)
        self.info = heap_info(self.h)
        self.base = int(self.info.data)

    def close(self):
        if self.h:
            heap_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def alloc(self, sizes, ptrs, stream=None):
        heap_alloc_batch(self.h, sizes, ptrs, stream=stream)

    def free(self, ptrs, sizes=None, status=None, stream=None):
        heap_free_batch(self.h, sizes, ptrs, stream=stream, status=status)

    def trim(self, stream=None):
        heap_trim(self.h, stream)

    def snapshot(self, stream=None) -> bytes:
        return heap_snapshot(self.h, stream)

    def error(self) -> int:
        return heap_get_error(self.h)

    def stats(self) -> dict:
        return heap_stats(self.h)

    def set_flags(self, flags: int):
        heap_set_flags(self.h, flags)

    def replay(self, ops, out, stream=None):
        heap_replay(self.h, ops, out, stream=stream)

    def pattern_write(self, ptrs, sizes, seed: int, stream=None):
        heap_pattern_write(self.h, ptrs, sizes, seed, stream=stream)

    def pattern_check(self, ptrs, sizes, seed: int, stream=None) -> int:
        import torch
        m = torch.zeros(1, dtype=torch.int64, device=ptrs.device)
        heap_pattern_check(self.h, ptrs, sizes, seed, m, stream=stream)
        return int(m.item())


class Growth:
    """Owns one growth run over a Heap; methods forward to the C ABI."""

    def __init__(self, heap: Heap, doublings, steps: int = 9, seed: int = 0):
        self.heap = heap
        self.agents = int(doublings.numel())
        self.g = growth_create(heap.h, self.agents, doublings, steps, seed)
        self.steps, self.seed = steps, seed

    def close(self):
        if self.g:
            growth_destroy(self.g)
            self.g = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, s: int, stream=None):
        growth_step(self.g, s, stream)

    def run_graph(self, stream=None):
        growth_graph_launch(self.g, stream)

    def release(self, stream=None):
        growth_release(self.g, stream)

    def export(self, stream=None):
        """(ptrs int64 tensor, bytes int64 tensor, failures int)."""
        import torch
        ptrs = torch.zeros(self.agents, dtype=torch.int64, device="cuda")
        nbytes = torch.zeros(self.agents, dtype=torch.int64, device="cuda")
        fails = torch.zeros(1, dtype=torch.int64, device="cuda")
        growth_export(self.g, ptrs, nbytes, fails, stream)
        return ptrs, nbytes, int(fails.item())

    def shape(self) -> tuple[int, int]:
        return growth_launch_shape(self.g)
