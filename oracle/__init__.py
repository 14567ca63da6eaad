"""CPU oracle of the device heap allocator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does, and this package imports nothing from it.

The C sources (``hbheap_oracle.c``, ``hbheap_model.c``) hold the oracle:

* a sequential allocator with the same size classes as the device heap
  (Introduction; Results, "Page allocator" and "Chunk allocator"), with two
  tie-break policies: LOWEST (canonical outcome) and FIFO (what a single
  device thread sees);
* an invariant checker for block lists and heap snapshots;
* the seeded payload pattern (MurmurHash3's 32-bit finaliser);
* a step-level model of the concurrent algorithm, explored exhaustively.

This module compiles them with gcc into ``liboracle.so`` and wraps them with
ctypes over numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["hbheap_oracle.c", "hbheap_model.c", "hbheap_shards_model.c", "hbheap_seg_model.c"]

VARIANT_CHUNK, VARIANT_PAGE, VARIANT_VA_PAGE, VARIANT_VA_CHUNK, VARIANT_VL_PAGE, VARIANT_VL_CHUNK = 0, 1, 2, 3, 4, 5
POLICY_LOWEST, POLICY_FIFO = 0, 1
FREE_OK, FREE_DOUBLE, FREE_INVALID, FREE_NULL = 0, 1, 2, 3
MAX_CLASSES = 16


def build(force: bool = True) -> str:
    """Compile the oracle's C sources into ``liboracle.so`` (gcc, -O2)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(s) for s in srcs + [os.path.join(HERE, "hbheap_oracle.h")])
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-g", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Acct(C.Structure):
    _fields_ = [
        ("n_classes", C.c_uint32), ("pad", C.c_uint32),
        ("n_chunks", C.c_uint64), ("free_chunks", C.c_uint64),
        ("live", C.c_uint64 * MAX_CLASSES), ("chunks", C.c_uint64 * MAX_CLASSES),
        ("free_pages", C.c_uint64 * MAX_CLASSES),
        ("n_alloc_ok", C.c_uint64), ("n_alloc_null", C.c_uint64), ("n_free_ok", C.c_uint64),
        ("n_free_double", C.c_uint64), ("n_free_invalid", C.c_uint64),
    ]


class BlocksReport(C.Structure):
    _fields_ = [
        ("n", C.c_uint64), ("n_null", C.c_uint64), ("n_nonnull", C.c_uint64),
        ("n_null_valid", C.c_uint64), ("n_bad_size_nonnull", C.c_uint64),
        ("n_oob", C.c_uint64), ("n_misaligned", C.c_uint64), ("n_straddle", C.c_uint64),
        ("n_overlap", C.c_uint64), ("live", C.c_uint64 * MAX_CLASSES),
    ]


class SnapReport(C.Structure):
    _fields_ = [
        ("ok_header", C.c_int32), ("n_classes", C.c_uint32),
        ("bad_class_byte", C.c_uint64), ("bad_free_chunk", C.c_uint64), ("bad_stray_bits", C.c_uint64),
        ("bad_count", C.c_uint64), ("bad_pool", C.c_uint64), ("bad_ring_ctl", C.c_uint64),
        ("bad_ring_entry", C.c_uint64), ("bad_ring_missing", C.c_uint64), ("bad_ring_dup", C.c_uint64),
        ("bad_conservation", C.c_uint64), ("bad_owned", C.c_uint64),
        ("bad_vdir", C.c_uint64), ("bad_vtaken", C.c_uint64), ("bad_vstore", C.c_uint64),
        ("bad_committed", C.c_uint64), ("free_chunks", C.c_uint64),
        ("live", C.c_uint64 * MAX_CLASSES), ("chunks", C.c_uint64 * MAX_CLASSES),
        ("free_pages", C.c_uint64 * MAX_CLASSES),
        ("stale_entries", C.c_uint64), ("eager", C.c_uint32), ("pad", C.c_uint32),
        ("whole_owned", C.c_uint64),
    ]

    def violations(self) -> dict:
        names = [f for f, _ in self._fields_ if f.startswith("bad_")]
        return {n: int(getattr(self, n)) for n in names if getattr(self, n)}


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB_PATH)
        u64, i64, u32, i32, vp = C.c_uint64, C.c_int64, C.c_uint32, C.c_int32, C.c_void_p
        sig = {
            "orc_class_of": (C.c_int, [u64, u64]),
            "orc_num_classes": (u32, [u64]),
            "orc_page_bytes": (u64, [u32]),
            "orc_pages_per_chunk": (u64, [u64, u32]),
            "orc_shard_geometry": (None, [u64, u32, C.POINTER(u32), C.POINTER(u32)]),
            "orc_page_ring_entries": (u64, [u64, u64, u32]),
            "orc_page_max_chunks": (u64, [u64, u64, u32, u32]),
            "orc_geometry_ok": (C.c_int, [u64, u64]),
            "orc_create": (vp, [u64, u64, C.c_int, C.c_int]),
            "orc_create_ex": (vp, [u64, u64, C.c_int, C.c_int, u32]),
            "orc_shards": (u32, [vp]),
            "orc_set_eager": (C.c_int, [vp]),
            "orc_destroy": (None, [vp]),
            "orc_alloc": (i64, [vp, u64]),
            "orc_free": (C.c_int, [vp, i64]),
            "orc_trim": (None, [vp]),
            "orc_alloc_batch": (None, [vp, vp, vp, u64]),
            "orc_free_batch": (None, [vp, vp, u64, vp]),
            "orc_accounting": (None, [vp, C.POINTER(Acct)]),
            "orc_replay": (None, [vp, vp, u64, vp]),
            "orc_fmix32": (u32, [u32]),
            "orc_pattern_word": (u32, [u32, u32, u32]),
            "orc_pattern_fill": (None, [u32, u32, vp, u64]),
            "orc_pattern_sum": (u32, [u32, u32, u64]),
            "orc_classes": (None, [vp, u64, u64, vp]),
            "orc_va_log2_seg": (u32, [u64, u64, u32]),
            "orc_va_segments": (u64, [u64, u64, u32]),
            "orc_va_budget": (u64, [u64, u64, u32]),
            "orc_va_chunk_log2_seg": (u32, [u64, u64, u32]),
            "orc_va_chunk_segments": (u64, [u64, u64, u32]),
            "orc_pattern_sums": (None, [u32, vp, vp, u64, vp]),
            "orc_check_blocks": (C.c_int, [u64, u64, vp, vp, u64, C.POINTER(BlocksReport)]),
            "orc_check_snapshot": (C.c_int, [vp, u64, C.POINTER(SnapReport)]),
            "orc_check_blocks_in_snapshot": (u64, [vp, u64, vp, vp, u64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _model_sigs(L)
        _lib = L
    return _lib


def _model_sigs(L):
    if not hasattr(L, "orc_model_run"):
        return
    L.orc_model_run.restype = C.c_int
    L.orc_model_run.argtypes = [C.POINTER(ModelParams), C.POINTER(ModelResult)]
    L.orc_shards_model_run.restype = C.c_int
    L.orc_shards_model_run.argtypes = [C.POINTER(ShardsParams), C.POINTER(ShardsResult)]
    L.orc_seg_model_run.restype = C.c_int
    L.orc_seg_model_run.argtypes = [C.POINTER(SegParams), C.POINTER(SegResult)]


class ShardsOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_int32), ("b", C.c_int32)]


class ShardsParams(C.Structure):
    _fields_ = [
        ("n_shards", C.c_int32), ("chunks", C.c_int32), ("ppc", C.c_int32), ("n_leaders", C.c_int32),
        ("ops", ShardsOp * 3), ("taken", C.c_int32 * 3), ("prealloc", C.c_uint32 * 3),
        ("mutation", C.c_int32), ("room", C.c_int32), ("max_states", C.c_int64),
    ]


class ShardsResult(C.Structure):
    _fields_ = [
        ("states", C.c_int64), ("terminals", C.c_int64), ("violations", C.c_int64), ("deadlocks", C.c_int64),
        ("oom_violations", C.c_int64), ("final_violations", C.c_int64), ("grant_violations", C.c_int64),
        ("null_outcomes", C.c_int64), ("truncated", C.c_int32), ("first_violation", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class SegOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("queue", C.c_int32), ("value", C.c_int32)]


class SegParams(C.Structure):
    _fields_ = [
        ("list", C.c_int32), ("n_queues", C.c_int32), ("segments", C.c_int32), ("n_leaders", C.c_int32),
        ("n_ops", C.c_int32 * 3), ("ops", (SegOp * 6) * 3), ("consume_all", C.c_int32), ("mutation", C.c_int32),
        ("max_states", C.c_int64),
    ]


class SegResult(C.Structure):
    _fields_ = [
        ("states", C.c_int64), ("terminals", C.c_int64), ("violations", C.c_int64), ("deadlocks", C.c_int64),
        ("value_violations", C.c_int64), ("segment_violations", C.c_int64), ("final_violations", C.c_int64),
        ("truncated", C.c_int32), ("first_violation", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


GOP_PUT, GOP_GET = 1, 2
SEG_MUTATIONS = {"close_early": 1, "install_blind": 2, "keep_count": 3, "retire_uncounted": 4, "link_early": 5}


def seg_model_run(list_form: bool, n_queues: int, segments: int, leaders: list, consume_all: bool = True,
                  mutation: int = 0, max_states: int = 3_000_000) -> dict:
    """Explore every interleaving of the leaders' operations (each a list of
    (GOP_PUT, queue, value) or (GOP_GET, queue)) on virtualised queues of
    2-slot segments drawn from a store of `segments` ids."""
    p = SegParams()
    p.list, p.n_queues, p.segments, p.n_leaders = int(list_form), n_queues, segments, len(leaders)
    for l, ops in enumerate(leaders):
        p.n_ops[l] = len(ops)
        for i, op in enumerate(ops):
            kind, q, v = (tuple(op) + (0,))[:3]
            p.ops[l][i] = SegOp(kind, q, v)
    p.consume_all, p.mutation, p.max_states = int(consume_all), mutation, max_states
    r = SegResult()
    rc = lib().orc_seg_model_run(C.byref(p), C.byref(r))
    if rc != 0:
        raise ValueError(f"bad segment model parameters ({rc})")
    return r.as_dict()


SOP_ALLOC, SOP_FREE = 1, 2
SHARDS_MUTATIONS = {"state_before_pool": 1, "ignore_positions": 2, "ignore_holds": 3, "home_only": 4,
                    "room_no_cap": 5, "room_keep_excess": 6, "room_back_all": 7}


def shards_model_run(n_shards: int, chunks: int, ppc: int, ops: list, taken=(0, 0, 0), prealloc=(0, 0, 0),
                     mutation: int = 0, room: int = 0, max_states: int = 4_000_000) -> dict:
    """Explore every interleaving of the leaders' operations (each
    (SOP_ALLOC, pages, home) or (SOP_FREE, first page, count)) on n_shards
    shards of `chunks` chunks of `ppc` pages; taken[j] chunks of shard j start
    owned by the class, with the pages in prealloc[j] allocated and the rest
    published; room > 0 caps the chunks the class may own per shard.
    Returns the counters."""
    p = ShardsParams()
    p.n_shards, p.chunks, p.ppc, p.n_leaders = n_shards, chunks, ppc, len(ops)
    for i, (kind, a, b) in enumerate(ops):
        p.ops[i] = ShardsOp(kind, a, b)
    for j in range(3):
        p.taken[j] = taken[j] if j < len(taken) else 0
        p.prealloc[j] = prealloc[j] if j < len(prealloc) else 0
    p.mutation, p.room, p.max_states = mutation, room, max_states
    r = ShardsResult()
    rc = lib().orc_shards_model_run(C.byref(p), C.byref(r))
    if rc != 0:
        raise ValueError(f"bad shards model parameters ({rc})")
    return r.as_dict()


class ModelOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("a", C.c_int32), ("b", C.c_int32)]


class ModelParams(C.Structure):
    _fields_ = [
        ("variant", C.c_int32), ("n_chunks", C.c_int32), ("ppc", C.c_int32), ("maxc", C.c_int32),
        ("n_leaders", C.c_int32), ("n_ops", C.c_int32 * 3), ("ops", (ModelOp * 3) * 3),
        ("prefill", C.c_int32), ("freeze", C.c_int32), ("mutation", C.c_int32), ("dry_hint", C.c_int32),
        ("fast_first", C.c_int32), ("first_nohold", C.c_int32), ("early_requeue", C.c_int32), ("pad2_", C.c_int32), ("max_states", C.c_int64),
    ]


class ModelResult(C.Structure):
    _fields_ = [
        ("states", C.c_int64), ("terminals", C.c_int64), ("violations", C.c_int64), ("deadlocks", C.c_int64),
        ("token_violations", C.c_int64), ("oom_violations", C.c_int64), ("final_violations", C.c_int64),
        ("grant_violations", C.c_int64), ("blocked_freezes", C.c_int64), ("null_outcomes", C.c_int64),
        ("truncated", C.c_int32), ("first_violation", C.c_int32), ("blocking_pcs", C.c_uint32),
        ("dry_starts", C.c_uint32), ("blocking_set", C.c_uint64 * 4),
    ]

    def as_dict(self) -> dict:
        d = {f: int(getattr(self, f)) for f, _ in self._fields_ if f not in ("pad", "blocking_set")}
        d["blocking_set"] = {64 * q + b for q in range(4) for b in range(64) if (self.blocking_set[q] >> b) & 1}
        return d


OP_ALLOC, OP_FREE_OWN, OP_FREE_GIVEN = 1, 2, 3
MUTATIONS = {"no_hold": 1, "requeue_always": 2, "free_enqueue_always": 3, "no_refund": 4,
             "release_no_publish": 5, "publish_early": 6, "dry_always": 7,
             "scan_no_positions": 8, "eager_exact_position": 9, "eager_no_stale_bit": 11}


def model_run(variant: int, n_chunks: int, ppc: int, leaders: list, prefill: int = 0, maxc: int | None = None,
              freeze: bool = False, mutation: int = 0, max_states: int = 2_000_000, dry_hint: bool = True,
              fast_first: bool = False, first_nohold: bool = True, early_requeue: bool = True) -> dict:
    """Explore every interleaving of `leaders` (each a list of (kind, a, b)
    ops) on a heap of n_chunks chunks of ppc pages.  Returns the counters."""
    p = ModelParams()
    p.variant, p.n_chunks, p.ppc = variant, n_chunks, ppc
    p.maxc = n_chunks if maxc is None else maxc
    p.n_leaders = len(leaders)
    for l, ops in enumerate(leaders):
        p.n_ops[l] = len(ops)
        for i, op in enumerate(ops):
            kind, a, b = (tuple(op) + (0, 0))[:3]
            p.ops[l][i] = ModelOp(kind, a, b)
    p.prefill, p.freeze, p.mutation, p.max_states = prefill, int(freeze), mutation, max_states
    p.dry_hint = int(dry_hint)
    p.fast_first = int(fast_first)
    p.first_nohold = int(first_nohold)
    p.early_requeue = int(early_requeue)
    r = ModelResult()
    rc = lib().orc_model_run(C.byref(p), C.byref(r))
    if rc != 0:
        raise ValueError(f"bad model parameters ({rc})")
    return r.as_dict()


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data) if a.size else C.c_void_p(0)


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------

def class_of(n: int, chunk_bytes: int) -> int:
    return int(lib().orc_class_of(n, chunk_bytes))


def classes(sizes: np.ndarray, chunk_bytes: int) -> np.ndarray:
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    out = np.empty(len(sizes), dtype=np.int8)
    lib().orc_classes(_ptr(sizes), len(sizes), chunk_bytes, _ptr(out))
    return out


def num_classes(chunk_bytes: int) -> int:
    return int(lib().orc_num_classes(chunk_bytes))


def page_bytes(k: int) -> int:
    return int(lib().orc_page_bytes(k))


def pages_per_chunk(chunk_bytes: int, k: int) -> int:
    return int(lib().orc_pages_per_chunk(chunk_bytes, k))


def shard_geometry(n_chunks: int, requested: int = 0) -> tuple[int, int]:
    """(shards, log2 span) for a heap of n_chunks chunks."""
    S, L = C.c_uint32(), C.c_uint32()
    lib().orc_shard_geometry(n_chunks, requested, C.byref(S), C.byref(L))
    return int(S.value), int(L.value)


def page_ring_entries(nbytes: int, chunk_bytes: int, shards: int = 1) -> int:
    return int(lib().orc_page_ring_entries(nbytes, chunk_bytes, shards))


def va_log2_seg(nbytes: int, chunk_bytes: int, shards: int = 1) -> int:
    return int(lib().orc_va_log2_seg(nbytes, chunk_bytes, shards))


def va_segments(nbytes: int, chunk_bytes: int, shards: int = 1) -> int:
    return int(lib().orc_va_segments(nbytes, chunk_bytes, shards))


def va_budget(nbytes: int, chunk_bytes: int, shards: int = 1) -> int:
    return int(lib().orc_va_budget(nbytes, chunk_bytes, shards))


def va_chunk_log2_seg(nbytes: int, chunk_bytes: int, shards: int = 0) -> int:
    """Virtualised array chunk variant; shards as requested of a heap (0 auto)."""
    return int(lib().orc_va_chunk_log2_seg(nbytes, chunk_bytes, shards))


def va_chunk_segments(nbytes: int, chunk_bytes: int, shards: int = 0) -> int:
    return int(lib().orc_va_chunk_segments(nbytes, chunk_bytes, shards))


def page_max_chunks(nbytes: int, chunk_bytes: int, k: int, shards: int = 1) -> int:
    """Chunks one class may own in one shard (page variant)."""
    return int(lib().orc_page_max_chunks(nbytes, chunk_bytes, k, shards))


# --------------------------------------------------------------------------
# sequential allocator
# --------------------------------------------------------------------------

class OracleHeap:
    """Sequential allocator; offsets from the data base, -1 for NULL."""

    def __init__(self, nbytes: int, chunk_bytes: int, variant: int = VARIANT_CHUNK, policy: int = POLICY_LOWEST,
                 shards: int = 1, eager: bool = False):
        self.h = lib().orc_create_ex(nbytes, chunk_bytes, variant, policy, shards)
        if not self.h:
            raise ValueError("invalid oracle geometry")
        if eager and lib().orc_set_eager(self.h) != 0:
            lib().orc_destroy(self.h)
            self.h = None
            raise ValueError("eager retirement needs the chunk variant")
        self.nbytes, self.chunk_bytes = nbytes, chunk_bytes
        self.n_chunks = nbytes // chunk_bytes
        self.variant, self.policy = variant, policy
        self.shards = int(lib().orc_shards(self.h))

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, n: int) -> int:
        return int(lib().orc_alloc(self.h, n))

    def free(self, off: int) -> int:
        return int(lib().orc_free(self.h, off))

    def trim(self):
        lib().orc_trim(self.h)

    def alloc_batch(self, sizes: np.ndarray) -> np.ndarray:
        sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
        out = np.empty(sizes.shape[0], dtype=np.int64)
        lib().orc_alloc_batch(self.h, _ptr(sizes), _ptr(out), sizes.shape[0])
        return out

    def free_batch(self, offs: np.ndarray) -> np.ndarray:
        offs = np.ascontiguousarray(offs, dtype=np.int64)
        st = np.empty(offs.shape[0], dtype=np.int32)
        lib().orc_free_batch(self.h, _ptr(offs), offs.shape[0], _ptr(st))
        return st

    def replay(self, ops: np.ndarray) -> np.ndarray:
        ops = np.ascontiguousarray(ops, dtype=np.int64)
        out = np.empty(ops.shape[0], dtype=np.int64)
        lib().orc_replay(self.h, _ptr(ops), ops.shape[0], _ptr(out))
        return out

    def accounting(self) -> dict:
        a = Acct()
        lib().orc_accounting(self.h, C.byref(a))
        K = a.n_classes
        return {
            "n_chunks": a.n_chunks, "free_chunks": a.free_chunks,
            "live": list(a.live)[:K], "chunks": list(a.chunks)[:K], "free_pages": list(a.free_pages)[:K],
            "n_alloc_ok": a.n_alloc_ok, "n_alloc_null": a.n_alloc_null, "n_free_ok": a.n_free_ok,
            "n_free_double": a.n_free_double, "n_free_invalid": a.n_free_invalid,
        }


# --------------------------------------------------------------------------
# pattern
# --------------------------------------------------------------------------

def fmix32(x: int) -> int:
    return int(lib().orc_fmix32(x & 0xFFFFFFFF))


def pattern_word(seed: int, req: int, i: int) -> int:
    return int(lib().orc_pattern_word(seed & 0xFFFFFFFF, req & 0xFFFFFFFF, i & 0xFFFFFFFF))


def pattern_bytes(seed: int, req: int, nbytes: int) -> bytes:
    buf = np.empty(nbytes, dtype=np.uint8)
    lib().orc_pattern_fill(seed & 0xFFFFFFFF, req & 0xFFFFFFFF, _ptr(buf), nbytes)
    return buf.tobytes()


def pattern_sum(seed: int, req: int, nbytes: int) -> int:
    return int(lib().orc_pattern_sum(seed & 0xFFFFFFFF, req & 0xFFFFFFFF, nbytes))


def pattern_sums(seed: int, reqs: np.ndarray, sizes: np.ndarray) -> np.ndarray:
    reqs = np.ascontiguousarray(reqs, dtype=np.uint64)
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    out = np.empty(len(reqs), dtype=np.uint32)
    lib().orc_pattern_sums(seed & 0xFFFFFFFF, _ptr(reqs), _ptr(sizes), len(reqs), _ptr(out))
    return out


# --------------------------------------------------------------------------
# checker
# --------------------------------------------------------------------------

def check_blocks(data_bytes: int, chunk_bytes: int, sizes: np.ndarray, offs: np.ndarray) -> BlocksReport:
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    rep = BlocksReport()
    lib().orc_check_blocks(data_bytes, chunk_bytes, _ptr(sizes), _ptr(offs), sizes.shape[0], C.byref(rep))
    return rep


def check_snapshot(snap: bytes | np.ndarray) -> SnapReport:
    a = np.frombuffer(bytes(snap), dtype=np.uint8) if not isinstance(snap, np.ndarray) else np.ascontiguousarray(snap, dtype=np.uint8)
    rep = SnapReport()
    lib().orc_check_snapshot(_ptr(a), a.shape[0], C.byref(rep))
    return rep


def check_blocks_in_snapshot(snap, sizes: np.ndarray, offs: np.ndarray) -> int:
    a = np.frombuffer(bytes(snap), dtype=np.uint8) if not isinstance(snap, np.ndarray) else np.ascontiguousarray(snap, dtype=np.uint8)
    sizes = np.ascontiguousarray(sizes, dtype=np.uint64)
    offs = np.ascontiguousarray(offs, dtype=np.int64)
    return int(lib().orc_check_blocks_in_snapshot(_ptr(a), a.shape[0], _ptr(sizes), _ptr(offs), sizes.shape[0]))
