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

VARIANT_CHUNK, VARIANT_PAGE = 0, 1
OK, E_INVAL, E_NOMEM, E_HIP, E_RANGE, E_UNSUP = 0, -1, -2, -3, -4, -5
ERR_DOUBLE_FREE, ERR_INVALID_FREE, ERR_TIMEOUT, ERR_CORRUPT = 0x1, 0x2, 0x4, 0x8
FLAG_STATS = 0x1
STAT_NAMES = ["chunk_grabs", "refills", "oom", "oom_waits", "double_free", "invalid_free", "timeouts", "reserved7",
              "state_ops", "headtail_ops", "pool_ops", "spread_ops", "reserved12", "reserved13", "reserved14",
              "reserved15"]
FREE_OK, FREE_DOUBLE, FREE_INVALID, FREE_NULL = 0, 1, 2, 3

EXPORTS = [
    "heap_create", "heap_create_ex", "heap_destroy", "heap_alloc_batch", "heap_free_batch", "heap_free_batch_ex",
    "heap_device_handle", "heap_set_flags", "heap_info", "heap_trim", "heap_snapshot", "heap_get_error", "heap_clear_error",
    "heap_stats", "heap_replay", "heap_pattern_write", "heap_pattern_check", "hb_atomic_probe", "hb_stream_copy",
    "hb_plain_set_heap", "hb_plain_alloc", "hb_plain_free", "hbheap_version",
]


class HbHeapError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} returned {code}")
        self.code = code


class HeapConfig(C.Structure):
    _fields_ = [("variant", C.c_uint32), ("width", C.c_uint32), ("spin_cap", C.c_uint32),
                ("backoff_max", C.c_uint32), ("flags", C.c_uint32), ("shards", C.c_uint32)]


class HeapInfo(C.Structure):
    _fields_ = [("data", C.c_void_p), ("data_bytes", C.c_uint64), ("chunk_bytes", C.c_uint64),
                ("n_chunks", C.c_uint64), ("n_classes", C.c_uint32), ("variant", C.c_uint32),
                ("ring_entries", C.c_uint64), ("state_bytes", C.c_uint64), ("metadata_bytes", C.c_uint64),
                ("n_shards", C.c_uint32), ("reserved", C.c_uint32)]


class DevHandle(C.Structure):
    """Mirror of hbheap_dev_t (passed by value to user kernels)."""
    _fields_ = [(n, C.c_void_p) for n in ("data", "state", "pool", "classes", "chunk_class", "chunk_cnt", "bits",
                                          "pool_ids", "slots", "err", "stats")] + \
               [("data_bytes", C.c_uint64)] + \
               [(n, C.c_uint32) for n in ("n_chunks", "log2_chunk", "n_classes", "variant", "words_per_chunk",
                                          "log2q", "width", "spin_cap", "backoff_max", "flags", "n_shards",
                                          "log2_span")]


_lib = None


def lib():
    """Load libhbheap.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no fallback")
    L = C.CDLL(LIB_PATH)
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
        "heap_stats": [vp, C.POINTER(C.c_uint64), sz],
        "heap_replay": [vp, i64p, i64p, sz, vp],
        "heap_pattern_write": [vp, vp, vp, sz, u32, vp],
        "heap_pattern_check": [vp, vp, vp, sz, u32, vp, vp],
        "hb_atomic_probe": [i32, vp, sz, sz, u32, u32, vp],
        "hb_stream_copy": [vp, vp, sz, vp],
        "hb_plain_set_heap": [sz],
        "hb_plain_alloc": [vp, vp, sz, vp],
        "hb_plain_free": [vp, sz, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = args
    L.hbheap_version.restype = C.c_char_p
    L.hbheap_version.argtypes = []
    _lib = L
    return L


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
                spin_cap: int = 0, backoff_max: int = 0, flags: int = 0, shards: int = 0) -> int:
    cfg = HeapConfig(variant, width, spin_cap, backoff_max, flags, shards)
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
    a = (C.c_uint64 * 16)()
    _check("heap_stats", lib().heap_stats(h, a, 16))
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


def hbheap_version() -> str:
    return lib().hbheap_version().decode()


# ---------------------------------------------------------------------------
# convenience owner of a heap handle
# ---------------------------------------------------------------------------

class Heap:
    """Owns one heap; methods forward to the C ABI above."""

    def __init__(self, nbytes: int, chunk_bytes: int = 8192, variant: int = VARIANT_CHUNK, width: int = 64,
                 spin_cap: int = 0, backoff_max: int = 0, flags: int = 0, shards: int = 0):
        self.h = heap_create(nbytes, chunk_bytes, variant, width, spin_cap, backoff_max, flags, shards)
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
