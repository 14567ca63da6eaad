"""Pins of the CPU oracle against what the paper and plain mathematics fix.

The paper prints no worked example, so the oracle is pinned by closed forms
(class map minimality, capacity N * C / s), textbook special cases (a single
class with no frees is a bump allocator; the page variant alone is a FIFO
free list), brute force on small inputs (an occupancy map over every byte),
exact accounting, and the published MurmurHash3 vectors for the payload
pattern.  Each test names the mistake it would catch.
"""
import functools
import os
import struct

import numpy as np
import pytest

import oracle as O
from paper_2504_18211_amd import inputs

KiB = 1024
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


# ---------------------------------------------------------------------------
# class map: smallest power-of-two page >= n, 16 B minimum (Results: queues
# are per power-of-two size; reading: 16 B smallest page)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("C", [4 * KiB, 8 * KiB, 16 * KiB, 32 * KiB, 64 * KiB])
def test_class_map_is_minimal_cover(C):
    K = O.num_classes(C)
    assert O.page_bytes(K - 1) == C, "largest class must be the whole chunk"
    assert O.class_of(0, C) == -1 and O.class_of(C + 1, C) == -1
    for n in range(1, C + 1):
        k = O.class_of(n, C)
        s = O.page_bytes(k)
        assert s >= n and s >= 16
        assert k == 0 or O.page_bytes(k - 1) < n, (n, k)
        assert s & (s - 1) == 0


def test_pages_per_chunk_closed_form():
    for C in [4 * KiB, 8 * KiB, 64 * KiB]:
        for k in range(O.num_classes(C)):
            assert O.pages_per_chunk(C, k) * O.page_bytes(k) == C


# ---------------------------------------------------------------------------
# capacity: a heap of N chunks serves exactly N * C / s pages of one class
# ---------------------------------------------------------------------------

def shard_caps(nbytes, C, variant, k, shards):
    """Pages of class k a heap can hold: per shard min(chunks, cap) * ppc."""
    N = nbytes // C
    S, L = O.shard_geometry(N, shards)
    tot = 0
    for j in range(S):
        nj = min(N, (j + 1) << L) - (j << L)
        cj = nj if variant == O.VARIANT_CHUNK else min(nj, O.page_max_chunks(nbytes, C, k, S))
        tot += cj * O.pages_per_chunk(C, k)
    return tot


@pytest.mark.parametrize("variant", [O.VARIANT_CHUNK, O.VARIANT_PAGE])
@pytest.mark.parametrize("policy", [O.POLICY_LOWEST, O.POLICY_FIFO])
@pytest.mark.parametrize("shards", [1, 4])
def test_single_class_capacity_exact(variant, policy, shards):
    C, nbytes = 8 * KiB, 40 * 8 * KiB + 123  # ragged tail of heap bytes is unused
    N = nbytes // C
    for k in [0, 3, 6, 9]:
        h = O.OracleHeap(nbytes, C, variant, policy, shards)
        s = O.page_bytes(k)
        expect = shard_caps(nbytes, C, variant, k, shards)
        if variant == O.VARIANT_CHUNK:
            assert expect == N * (C // s)
        offs = h.alloc_batch(np.full(expect + 5, s, dtype=np.uint64))
        assert (offs[:expect] >= 0).all()
        assert (offs[expect:] < 0).all()
        a = h.accounting()
        assert a["live"][k] == expect and a["free_pages"][k] == 0
        h.close()


def test_shard_geometry_closed_form():
    for N in [1, 7, 32, 1000, 1024, 8192, 1 << 19, 1 << 21]:
        for req in [0, 1, 2, 8, 64]:
            S, L = O.shard_geometry(N, req)
            assert (S - 1) << L < N <= S << L, (N, req, S, L)
            want = req or min(64, max(1, 1 << ((N // 256).bit_length() - 1))) if N >= 256 else (req or 1)
            want = min(want, N)
            assert (1 << L) >= -(-N // want) and (L == 0 or (1 << (L - 1)) < -(-N // want))


def test_fifo_home_shard_then_steal():
    """One lane, two shards of two 8 KiB chunks: shard 0's queue, then its
    pool, then shard 1; a page freed in shard 0 is reused before shard 1."""
    C = 8 * KiB
    h = O.OracleHeap(4 * C, C, O.VARIANT_CHUNK, O.POLICY_FIFO, 2)
    assert h.shards == 2
    offs = [h.alloc(4096) for _ in range(5)]
    assert offs == [0, 4096, C, C + 4096, 2 * C]
    h.free(4096)
    assert h.alloc(4096) == 4096
    assert h.alloc(4096) == 2 * C + 4096
    h.close()


def test_lowest_single_class_is_bump_allocator():
    """No frees, one class, LOWEST policy: block i sits at i * s."""
    C, nbytes = 8 * KiB, 16 * 8 * KiB
    for s in [16, 48, 1000, 4096, 8192]:
        h = O.OracleHeap(nbytes, C)
        k = O.class_of(s, C)
        ps = O.page_bytes(k)
        n = nbytes // ps
        offs = h.alloc_batch(np.full(n, s, dtype=np.uint64))
        assert np.array_equal(offs, np.arange(n, dtype=np.int64) * ps)
        h.close()


def test_page_variant_fifo_is_a_fifo_free_list():
    """Page variant, FIFO policy, one class: after the fresh pages run out,
    allocations return freed pages in the order they were freed."""
    C, nbytes = 8 * KiB, 4 * 8 * KiB
    h = O.OracleHeap(nbytes, C, O.VARIANT_PAGE, O.POLICY_FIFO)
    ps = 1024
    n = nbytes // ps
    offs = h.alloc_batch(np.full(n, ps, dtype=np.uint64))
    assert np.array_equal(offs, np.arange(n) * ps)
    order = np.random.default_rng(5).permutation(n)
    for i in order:
        assert h.free(int(offs[i])) == O.FREE_OK
    again = h.alloc_batch(np.full(n, ps, dtype=np.uint64))
    assert np.array_equal(again, offs[order])
    h.close()


def test_chunk_variant_fifo_single_chunk_is_lowest_free_bit():
    """One chunk, chunk variant, FIFO policy: each allocation takes the lowest
    free page of that chunk (the scan inside a chunk)."""
    C = 8 * KiB
    h = O.OracleHeap(C, C, O.VARIANT_CHUNK, O.POLICY_FIFO)
    ps = 64
    n = C // ps
    offs = h.alloc_batch(np.full(n, ps, dtype=np.uint64))
    freed = sorted(np.random.default_rng(1).choice(n, 37, replace=False).tolist(), reverse=True)
    for i in freed:
        assert h.free(int(offs[i])) == O.FREE_OK
    again = h.alloc_batch(np.full(len(freed), ps, dtype=np.uint64))
    assert again.tolist() == sorted(int(offs[i]) for i in freed)
    h.close()


def test_chunk_variant_fifo_rotates_partial_chunks():
    """Two partially used chunks: a chunk that keeps free pages after serving
    goes to the back of its queue, so consecutive allocations alternate."""
    C = 8 * KiB
    h = O.OracleHeap(2 * C, C, O.VARIANT_CHUNK, O.POLICY_FIFO)
    ps = 1024  # 8 pages per chunk
    offs = h.alloc_batch(np.full(16, ps, dtype=np.uint64))
    # free pages 1,2 of chunk 0 then pages 3,4 of chunk 1
    for i in [1, 2, 8 + 3, 8 + 4]:
        h.free(int(offs[i]))
    again = h.alloc_batch(np.full(4, ps, dtype=np.uint64))
    assert again.tolist() == [1 * ps, C + 3 * ps, 2 * ps, C + 4 * ps]
    h.close()


# ---------------------------------------------------------------------------
# brute force: random mixed streams on a small heap against a byte map
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [O.VARIANT_CHUNK, O.VARIANT_PAGE])
@pytest.mark.parametrize("policy", [O.POLICY_LOWEST, O.POLICY_FIFO])
@pytest.mark.parametrize("seed,shards", [(1, 1), (2, 1), (3, 4), (4, 8)])
def test_random_stream_against_byte_map(variant, policy, seed, shards):
    C, nbytes = 4 * KiB, 24 * 4 * KiB
    h = O.OracleHeap(nbytes, C, variant, policy, shards)
    S, L = O.shard_geometry(nbytes // C, shards)
    occ = np.zeros(nbytes, dtype=np.int32)  # owner id + 1
    owner = {}                               # chunk -> class (no trim: owned for good)
    live = {}
    g = np.random.default_rng(seed)
    for step in range(4000):
        if live and g.random() < 0.45:
            rid = list(live)[int(g.integers(len(live)))]
            off, s = live.pop(rid)
            assert h.free(off) == O.FREE_OK
            assert (occ[off:off + s] == rid + 1).all()
            occ[off:off + s] = 0
        else:
            n = int(g.integers(1, C + 1)) if g.random() < 0.3 else int(g.integers(1, 200))
            off = h.alloc(n)
            k = O.class_of(n, C)
            if off < 0:
                # NULL only when no free page of the class exists and no shard
                # has an unowned chunk the class may still take (exact OOM)
                a = h.accounting()
                assert a["free_pages"][k] == 0
                for j in range(S):
                    chunks = range(j << L, min(nbytes // C, (j + 1) << L))
                    unowned = sum(1 for c in chunks if c not in owner)
                    mine = sum(1 for c in chunks if owner.get(c) == k)
                    capped = variant == O.VARIANT_PAGE and mine >= O.page_max_chunks(nbytes, C, k, S)
                    assert unowned == 0 or capped, (j, unowned, mine)
                continue
            s = O.page_bytes(k)
            assert off % s == 0 and off // C == (off + s - 1) // C and off + s <= (nbytes // C) * C
            assert (occ[off:off + s] == 0).all(), "overlap"
            assert owner.setdefault(off // C, k) == k, "chunk serves two classes"
            occ[off:off + s] = step + 1
            live[step] = (off, s)
    a = h.accounting()
    for k in range(O.num_classes(C)):
        assert a["live"][k] == sum(1 for (o, s) in live.values() if s == O.page_bytes(k))
    h.close()


def test_free_semantics():
    C = 8 * KiB
    h = O.OracleHeap(4 * C, C)
    a = h.alloc(100)  # 128 B class
    assert a == 0
    assert h.free(-1) == O.FREE_NULL
    assert h.free(a + 16) == O.FREE_INVALID  # misaligned for 128 B pages
    assert h.free(3 * C) == O.FREE_INVALID   # unowned chunk
    assert h.free(4 * C) == O.FREE_INVALID   # out of range
    before = h.accounting()
    assert h.free(a) == O.FREE_OK
    assert h.free(a) == O.FREE_DOUBLE        # double free changes nothing
    assert h.free(a + 128) == O.FREE_DOUBLE  # never-allocated page of an owned chunk is free
    after = h.accounting()
    assert after["live"][3] == before["live"][3] - 1
    assert after["n_free_double"] == 2 and after["n_free_invalid"] == 3
    h.close()


@pytest.mark.parametrize("variant", [O.VARIANT_CHUNK, O.VARIANT_PAGE])
@pytest.mark.parametrize("policy", [O.POLICY_LOWEST, O.POLICY_FIFO])
def test_trim_returns_to_fresh(variant, policy):
    C, nbytes = 8 * KiB, 64 * 8 * KiB
    sizes = inputs.sizes_log_uniform(3000, 4, 8 * KiB, 11)
    fresh = O.OracleHeap(nbytes, C, variant, policy)
    ref = fresh.alloc_batch(sizes)
    fresh.close()
    h = O.OracleHeap(nbytes, C, variant, policy)
    offs = h.alloc_batch(sizes)
    assert np.array_equal(offs, ref)
    st = h.free_batch(offs[::-1].copy())
    assert ((st == O.FREE_OK) | (st == O.FREE_NULL)).all()
    h.trim()
    a = h.accounting()
    assert a["free_chunks"] == nbytes // C and sum(a["chunks"]) == 0 and sum(a["live"]) == 0
    # a trimmed empty heap behaves exactly like a fresh one
    assert np.array_equal(h.alloc_batch(sizes), ref)
    h.close()


def test_replay_matches_stepwise_calls():
    ops = inputs.op_script(2000, 3, p_invalid_size=0.05)
    C, nbytes = 8 * KiB, 32 * 8 * KiB
    h1 = O.OracleHeap(nbytes, C, O.VARIANT_CHUNK, O.POLICY_FIFO)
    out = h1.replay(ops)
    h2 = O.OracleHeap(nbytes, C, O.VARIANT_CHUNK, O.POLICY_FIFO)
    ref = []
    for i, op in enumerate(ops):
        ref.append(h2.alloc(int(op)) if op >= 0 else h2.free(int(ref[-op - 1])))
    assert out.tolist() == ref


# ---------------------------------------------------------------------------
# checker: planted mistakes must be caught
# ---------------------------------------------------------------------------

def test_check_blocks_catches_planted_faults():
    C, data = 8 * KiB, 8 * 8 * KiB
    sizes = np.array([16, 16, 100, 8192, 0, 17], dtype=np.uint64)
    good = np.array([0, 16, 128, C, -1, 32], dtype=np.int64)
    r = O.check_blocks(data, C, sizes, good)
    assert r.n_overlap == 0 and r.n_misaligned == 0 and r.n_oob == 0 and r.n_null_valid == 0
    assert list(r.live)[:3] == [2, 1, 0] and r.live[3] == 1 and r.live[9] == 1
    bad = good.copy(); bad[1] = 8            # overlaps block 0, misaligned
    r = O.check_blocks(data, C, sizes, bad)
    assert r.n_overlap == 1 and r.n_misaligned == 1
    bad = good.copy(); bad[3] = 7 * C + 4096  # 8 KiB page straddles the heap end
    assert O.check_blocks(data, C, sizes, bad).n_oob == 1
    bad = good.copy(); bad[4] = 0             # non-NULL for a size-0 request
    assert O.check_blocks(data, C, sizes, bad).n_bad_size_nonnull == 1
    bad = good.copy(); bad[0] = -1            # NULL for a valid request
    assert O.check_blocks(data, C, sizes, bad).n_null_valid == 1
    bad = good.copy(); bad[2] = C - 64        # 128 B page at C-64 crosses into the next chunk
    r = O.check_blocks(data, C, sizes, bad)
    assert r.n_straddle == 1 and r.n_misaligned == 1


# ---------------------------------------------------------------------------
# snapshot checker on hand-built snapshots of the documented layout
# ---------------------------------------------------------------------------

def build_snapshot(N, log2C, variant, log2q, cls, cnt, bits, pool_bumps, pool_ids, rings, owned=None, S=1,
                   log2_span=None, va=None):
    """Write a version-4 snapshot from plain arrays (bitmask words
    word-major: word w of chunk c at index w*N + c).  rings[(j, k)] or
    rings[k] (shard 0) = (H, head, entries); pool_bumps: one per shard;
    pool_ids: the whole id array.  Virtualised array (variants 2 and 3):
    va = dict(g, ldir, lstore, M, budget, committed per shard); the slot
    region is the shards' M segments of 2^g slots; each queue's segments are
    numbered from the shard's first, queue after queue, the store holds the
    rest in ascending order."""
    K = log2C - 3
    W = (1 << log2C) // 1024
    Q = 1 << log2q
    if log2_span is None:
        log2_span = max(0, (N - 1).bit_length())
    if isinstance(pool_bumps, int):
        pool_bumps = [pool_bumps]

    def al(x):
        return (x + 255) & ~255
    off_pool = 256
    off_cl = al(off_pool + 128 * S)
    off_cls = al(off_cl + 512 * S * K)
    off_cnt = al(off_cls + N)
    off_bits = al(off_cnt + 4 * N)
    off_pid = al(off_bits + 8 * N * W)
    off_sl = al(off_pid + 4 * N)
    nslots = (S * va["M"]) << va["g"] if va else S * K * Q
    total = al(off_sl + 4 * nslots)
    vl = bool(va and va.get("vl"))
    if va:
        g, ldir, lstore, M = va["g"], va["ldir"], va["lstore"], va["M"]
        off_vdir = total
        off_vtk = al(off_vdir + 8 * (2 * S * M if vl else S * K * (1 << ldir)))
        off_vst = al(off_vtk + 4 * S * M)
        off_vss = al(off_vst + 512 * S)
        total = al(off_vss + 4 * S * (1 << lstore))
    b = bytearray(total)
    struct.pack_into("<IIQIIIIIIIIQQQQQQQQ", b, 0, 0x48424850, 4, N << log2C, N, log2C, K, variant, W, log2q,
                     S, log2_span, off_pool, off_cl, off_cls, off_cnt, off_bits, off_pid, off_sl, total)
    if va:
        struct.pack_into("<IIIIQQQQQ", b, 112, g, ldir, lstore, M, va["budget"], off_vdir, off_vtk, off_vst, off_vss)
    for j in range(S):
        first = j << log2_span
        size = min(N, (j + 1) << log2_span) - first
        struct.pack_into("<QII", b, off_pool + 128 * j, pool_bumps[j], size, first)
    for i, c in enumerate(pool_ids):
        struct.pack_into("<I", b, off_pid + 4 * i, c)
    b[off_cls:off_cls + N] = bytes(cls)
    for c in range(N):
        struct.pack_into("<I", b, off_cnt + 4 * c, cnt[c])
        for w in range(W):
            struct.pack_into("<Q", b, off_bits + 8 * (w * N + c), bits[c][w])
    rings = {(key if isinstance(key, tuple) else (0, key)): v for key, v in rings.items()}
    owned = {(key if isinstance(key, tuple) else (0, key)): v for key, v in (owned or {}).items()}
    for j in range(S):
        for k in range(K):
            r = j * K + k
            H, head, ents = rings.get((j, k), (0, 0, []))
            struct.pack_into("<Q", b, off_cl + 512 * r, (H << 32) | ((len(ents) + 0x80000000) & 0xFFFFFFFF))
            struct.pack_into("<I", b, off_cl + 512 * r + 128, head & 0xFFFFFFFF)
            struct.pack_into("<I", b, off_cl + 512 * r + 256, (head + len(ents)) & 0xFFFFFFFF)
            struct.pack_into("<Q", b, off_cl + 512 * r + 384, owned.get((j, k), 0))
            if va:
                continue
            for q in range(Q):
                struct.pack_into("<I", b, off_sl + 4 * (r * Q + q), 0xFFFFFFFF)
            for q, e in enumerate(ents):
                struct.pack_into("<I", b, off_sl + 4 * (r * Q + ((head + q) % Q)), e)
    if va:
        G, D, QS = 1 << g, 1 << ldir, 1 << lstore
        for i in range(S * M * G):
            struct.pack_into("<I", b, off_sl + 4 * i, 0xFFFFFFFF)
        for i in range(2 * S * M if vl else S * K * D):
            struct.pack_into("<Q", b, off_vdir + 8 * i, (1 << 64) - 1)
        for j in range(S):
            nxt = 0
            for k in range(K):
                r = j * K + k
                H, head, ents = rings.get((j, k), (0, 0, []))
                tail = head + len(ents)
                sg = head >> g
                if vl:
                    # a chain from the front (head's segment) to the back (the
                    # last written position's, the front if none)
                    last = max(sg, (tail - 1) >> g) if tail > 0 else sg
                    ids = list(range(nxt, nxt + last - sg + 1))
                    nxt += len(ids)
                    for i, m in enumerate(ids):
                        sn = sg + i
                        struct.pack_into("<Q", b, off_vdir + 8 * (j * M + m), (k << 32) | sn)
                        struct.pack_into("<Q", b, off_vdir + 8 * (S * M + j * M + m),
                                         ids[i + 1] if i + 1 < len(ids) else (1 << 64) - 1)
                        s0 = sn << g
                        struct.pack_into("<I", b, off_vtk + 4 * (j * M + m), max(0, min(head, s0 + G) - s0) if i == 0 else 0)
                        for p_ in range(max(s0, head), min(s0 + G, tail)):
                            struct.pack_into("<I", b, off_sl + 4 * (((j * M + m) << g) + (p_ - s0)), ents[p_ - head])
                    struct.pack_into("<QQ", b, off_cl + 512 * r + 392, (sg << 32) | ids[0], (last << 32) | ids[-1])
                    continue
                while (sg << g) < tail:
                    m = nxt
                    nxt += 1
                    struct.pack_into("<Q", b, off_vdir + 8 * ((r << ldir) + (sg & (D - 1))), ((sg & 0xFFFFFFFF) << 32) | m)
                    s0 = sg << g
                    struct.pack_into("<I", b, off_vtk + 4 * (j * M + m), max(0, min(head, s0 + G) - s0))
                    for p in range(max(s0, head), min(s0 + G, tail)):
                        struct.pack_into("<I", b, off_sl + 4 * (((j * M + m) << g) + (p - s0)), ents[p - head])
                    sg += 1
            free_ids = list(range(nxt, M))
            struct.pack_into("<QII", b, off_vst + 512 * j, len(free_ids) + 0x80000000, 0, 0)
            struct.pack_into("<I", b, off_vst + 512 * j + 128, 0)
            struct.pack_into("<I", b, off_vst + 512 * j + 256, len(free_ids))
            struct.pack_into("<Q", b, off_vst + 512 * j + 384, va["committed"][j])
            for i in range(QS):
                struct.pack_into("<I", b, off_vss + 4 * ((j << lstore) + i), free_ids[i] if i < len(free_ids) else 0xFFFFFFFF)
    return bytes(b)


def _tiny_state():
    # 4 chunks of 4 KiB (W = 4 words, K = 9); chunk 0 class 6 (1 KiB, 4 pages)
    # with pages 1,3 free; chunk 2 class 0 (16 B, 256 pages) with page 5 free;
    # chunks 1 and 3 unowned and still in the pool.
    N, log2C = 4, 12
    cls = [6, 0xFF, 0, 0xFF]
    cnt = [2, 0, 1, 0]
    bits = [[0b1010, 0, 0, 0], [0, 0, 0, 0], [1 << 5, 0, 0, 0], [0, 0, 0, 0]]
    pool_ids = [0, 2, 1, 3]     # consumed: 0, 2; left: 1, 3
    return N, log2C, cls, cnt, bits, pool_ids


def test_snapshot_checker_accepts_consistent_state():
    N, log2C, cls, cnt, bits, pool_ids = _tiny_state()
    snap = build_snapshot(N, log2C, 0, 2, cls, cnt, bits, 2, pool_ids, {6: (0, 5, [0]), 0: (0, 0, [2])})
    r = O.check_snapshot(snap)
    assert r.ok_header and not r.violations(), r.violations()
    assert r.free_chunks == 2 and r.live[6] == 2 and r.live[0] == 255 and r.free_pages[6] == 2


@pytest.mark.parametrize("plant,field", [
    ("count", "bad_count"), ("stray", "bad_stray_bits"), ("dup", "bad_ring_dup"),
    ("missing", "bad_ring_missing"), ("held", "bad_ring_ctl"), ("pool", "bad_pool"),
    ("freebits", "bad_free_chunk"), ("badclass", "bad_class_byte"),
])
def test_snapshot_checker_catches_planted_faults(plant, field):
    N, log2C, cls, cnt, bits, pool_ids = _tiny_state()
    rings = {6: (0, 5, [0]), 0: (0, 0, [2])}
    bump = 2
    if plant == "count":
        cnt[0] = 3
    elif plant == "stray":
        bits[0][0] |= 1 << 4           # class 6 has 4 pages per 4 KiB chunk
    elif plant == "dup":
        rings[6] = (0, 5, [0, 0])
    elif plant == "missing":
        rings[0] = (0, 0, [])
    elif plant == "held":
        rings[6] = (1, 5, [0])
    elif plant == "pool":
        pool_ids = [0, 1, 3, 3]
    elif plant == "freebits":
        bits[1][2] = 1
    elif plant == "badclass":
        cls[1] = 12
    snap = build_snapshot(N, log2C, 0, 2, cls, cnt, bits, bump, pool_ids, rings)
    v = O.check_snapshot(snap).violations()
    assert v.get(field, 0) > 0, (plant, v)


def test_snapshot_checker_page_variant():
    N, log2C, cls, cnt, bits, pool_ids = _tiny_state()
    # page variant: entries are byte offsets / 16 of the free pages; a ring of
    # 2^8 entries lets class 0 (256 pages per 4 KiB chunk) own one chunk
    e6 = [(0 * 4096 + 1 * 1024) // 16, (0 * 4096 + 3 * 1024) // 16]
    e0 = [(2 * 4096 + 5 * 16) // 16]
    snap = build_snapshot(N, log2C, 1, 8, cls, [0] * 4, bits, 2, pool_ids, {6: (0, 3, e6), 0: (0, 0, e0)},
                          owned={6: 1, 0: 1})
    assert not O.check_snapshot(snap).violations()
    bad = build_snapshot(N, log2C, 1, 8, cls, [0] * 4, bits, 2, pool_ids, {6: (0, 3, e6[:1]), 0: (0, 0, e0)},
                         owned={6: 1, 0: 1})
    assert O.check_snapshot(bad).violations().get("bad_ring_missing", 0) == 1
    bad = build_snapshot(N, log2C, 1, 8, cls, [0] * 4, bits, 2, pool_ids, {6: (0, 3, e6), 0: (0, 0, e0)},
                         owned={6: 2, 0: 1})
    assert O.check_snapshot(bad).violations().get("bad_owned", 0) == 1


def test_snapshot_checker_shards():
    """Two shards of two chunks: entries must stay inside their shard."""
    N, log2C, cls, cnt, bits, _ = _tiny_state()
    # shard 0 = chunks 0,1 (chunk 0 class 6, chunk 1 unowned); shard 1 = chunks 2,3
    pool_ids = [0, 1, 2, 3]
    good = build_snapshot(N, log2C, 0, 1, cls, cnt, bits, [1, 1], pool_ids, {(0, 6): (0, 0, [0]), (1, 0): (0, 0, [2])},
                          S=2, log2_span=1)
    assert not O.check_snapshot(good).violations(), O.check_snapshot(good).violations()
    bad = build_snapshot(N, log2C, 0, 1, cls, cnt, bits, [1, 1], pool_ids, {(0, 6): (0, 0, [0]), (0, 0): (0, 0, [2])},
                         S=2, log2_span=1)
    v = O.check_snapshot(bad).violations()
    assert v.get("bad_ring_entry", 0) == 1 and v.get("bad_ring_missing", 0) == 1
    bad = build_snapshot(N, log2C, 0, 1, cls, cnt, bits, [1, 0], [0, 1, 3, 2], {(0, 6): (0, 0, [0]), (1, 0): (0, 0, [2])},
                         S=2, log2_span=1)
    assert O.check_snapshot(bad).violations().get("bad_pool", 0) > 0


def test_blocks_in_snapshot():
    N, log2C, cls, cnt, bits, pool_ids = _tiny_state()
    snap = build_snapshot(N, log2C, 0, 2, cls, cnt, bits, 2, pool_ids, {6: (0, 5, [0]), 0: (0, 0, [2])})
    sizes = np.array([1000, 1000, 16, 16, 16], dtype=np.uint64)
    assert O.check_blocks_in_snapshot(snap, sizes, np.array([0, 2048, 2 * 4096, -1, 2 * 4096 + 16], dtype=np.int64)) == 0
    # page 1 of chunk 0 is free -> not a live block; 16 B block in a 1 KiB chunk
    assert O.check_blocks_in_snapshot(snap, sizes, np.array([1024, 0, 16, -1, -1], dtype=np.int64)) == 2


# ---------------------------------------------------------------------------
# payload pattern: MurmurHash3 x86_32 published vectors pin fmix32
# ---------------------------------------------------------------------------

def _rotl(x, r):
    return ((x << r) | (x >> (32 - r))) & 0xFFFFFFFF


def _murmur3_x86_32(key: bytes, seed: int) -> int:
    h, c1, c2 = seed, 0xCC9E2D51, 0x1B873593
    nb = len(key) // 4
    for i in range(nb):
        k = int.from_bytes(key[4 * i:4 * i + 4], "little")
        k = _rotl((k * c1) & 0xFFFFFFFF, 15) * c2 & 0xFFFFFFFF
        h = (_rotl(h ^ k, 13) * 5 + 0xE6546B64) & 0xFFFFFFFF
    t = key[4 * nb:]
    k = 0
    for j in range(len(t) - 1, -1, -1):
        k ^= t[j] << (8 * j)
    if t:
        h ^= _rotl((k * c1) & 0xFFFFFFFF, 15) * c2 & 0xFFFFFFFF
    return O.fmix32(h ^ len(key))


def test_fmix32_published_vectors():
    n = 0
    with open(os.path.join(GOLD, "murmur3_x86_32_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, seed, want = line.split()
            kb = b"" if key == "-" else bytes.fromhex(key)
            assert _murmur3_x86_32(kb, int(seed, 16)) == int(want, 16), line
            n += 1
    assert n >= 10


def test_pattern_bytes_little_endian_truncated():
    seed, req = 0xC0F2 ^ 77, 77
    w0, w1 = O.pattern_word(seed, req, 0), O.pattern_word(seed, req, 1)
    assert O.pattern_word(seed, req, 0) == O.fmix32(seed ^ O.fmix32(req) ^ 0)
    assert O.pattern_word(seed, req, 1) == O.fmix32(seed ^ O.fmix32(req) ^ 0x9E3779B9)
    b = O.pattern_bytes(seed, req, 6)
    assert b == w0.to_bytes(4, "little") + w1.to_bytes(4, "little")[:2]


def test_pattern_sum_against_bytes():
    """The block checksum is the wrap-around sum of the block's little-endian
    words, a partial last word zero-extended: closed forms at 0 and 4 bytes,
    and brute force from the pattern bytes for ragged sizes."""
    assert O.pattern_sum(7, 9, 0) == 0
    for seed, req in [(0, 0), (0xC0F5, 12345), (0xFFFFFFFF, 1 << 31)]:
        assert O.pattern_sum(seed, req, 4) == O.pattern_word(seed, req, 0)
        for n in [1, 2, 3, 5, 15, 16, 17, 63, 1000, 1021, 8192]:
            b = O.pattern_bytes(seed, req, n) + b"\0" * (-n % 4)
            expect = int(np.frombuffer(b, dtype="<u4").astype(np.uint64).sum() & 0xFFFFFFFF)
            assert O.pattern_sum(seed, req, n) == expect, (seed, req, n)
    reqs = np.array([1, 2, 3, 4], dtype=np.uint64)
    sizes = np.array([16, 5, 0, 4096], dtype=np.uint64)
    got = O.pattern_sums(99, reqs, sizes)
    assert got.tolist() == [O.pattern_sum(99, int(r), int(s)) for r, s in zip(reqs, sizes)]


def test_classes_batch_matches_scalar():
    sizes = np.array([0, 1, 15, 16, 17, 32, 33, 4096, 4097, 8192, 8193, 1 << 40], dtype=np.uint64)
    assert O.classes(sizes, 8192).tolist() == [O.class_of(int(s), 8192) for s in sizes]



# ---------------------------------------------------------------------------
# virtualised array page variant: budget closed form, capacity, snapshots
# ---------------------------------------------------------------------------

def test_va_budget_closed_form():
    """Segments of 2^g entries, g = log2(Q) - 3 within [4, 10]; M = K*Q/2^g
    per shard; the shard's classes may own (M - 3K) * 2^g pages."""
    for nbytes, C, S in [(4 << 30, 8192, 64), (8 << 20, 8192, 2), (64 << 20, 16384, 4), (1 << 20, 4096, 1)]:
        K = O.num_classes(C)
        Q = O.page_ring_entries(nbytes, C, S)
        g = min(10, max(4, Q.bit_length() - 1 - 3))
        M = (K * Q) >> g
        assert O.va_log2_seg(nbytes, C, S) == g
        assert O.va_segments(nbytes, C, S) == M
        assert O.va_budget(nbytes, C, S) == (max(0, M - 3 * K) << g)


def test_va_capacity_is_shared_by_the_classes_of_a_shard():
    """One class alone can use the whole shard budget (the page variant caps
    each class at Q entries); with two classes the budget is shared."""
    nbytes, C = 2 << 20, 8192          # 256 chunks, one shard
    budget = O.va_budget(nbytes, C, 1)
    Q = O.page_ring_entries(nbytes, C, 1)
    va = O.OracleHeap(nbytes, C, O.VARIANT_VA_PAGE)
    pg = O.OracleHeap(nbytes, C, O.VARIANT_PAGE)
    n16 = 0
    while va.alloc(16) >= 0:
        n16 += 1
    m16 = 0
    while pg.alloc(16) >= 0:
        m16 += 1
    ppc = 512
    assert n16 == min(256, budget // ppc) * ppc
    assert m16 == min(256, Q // ppc) * ppc
    assert n16 > m16
    # the budget is in pages: a second class gets what the first left
    nbig = 0
    while va.alloc(4096) >= 0:
        nbig += 1
    used = (n16 // ppc) * ppc
    assert nbig == min(256 - n16 // ppc, (budget - used) // 2) * 2


def _va_state(tamper=None):
    # one shard, 4 chunks of 4 KiB (K = 9, W = 4): chunk 0 class 6 (1 KiB, 4
    # pages) with pages 1 and 3 free, chunk 2 class 0 with page 5 free;
    # segments of 16 entries, 64 segments, directory 128, store 64
    N, log2C, K = 4, 12, 9
    cls = [6, 0xFF, 0, 0xFF]
    cnt = [2, 0, 1, 0]
    bits = [[0] * 4 for _ in range(N)]
    bits[0][0] = (1 << 1) | (1 << 3)
    bits[2][0] = 1 << 5
    off = lambda c, k, p: ((c << log2C) + p * (16 << k)) >> 4
    rings = {6: (0, 30, [off(0, 6, 1), off(0, 6, 3)]), 0: (0, 16, [off(2, 0, 5)])}
    owned = {6: 1, 0: 1}
    committed = [4 + 256]
    va = dict(g=4, ldir=7, lstore=6, M=64, budget=(64 - 27) << 4, committed=committed)
    if tamper:
        tamper(rings, owned, va)
    return build_snapshot(N, log2C, 2, 7, cls, cnt, bits, [2], [0, 2, 1, 3], rings, owned=owned, va=va)


def test_va_snapshot_clean_and_planted_faults():
    rep = O.check_snapshot(_va_state())
    assert rep.ok_header and not rep.violations(), rep.violations()
    b = bytearray(_va_state())
    off_vdir, off_vtk, off_vst, off_vss = struct.unpack_from("<QQQQ", b, 136)
    off_sl = struct.unpack_from("<Q", b, 96)[0]
    # a directory entry naming the wrong segment number
    x = bytearray(b)
    ring6 = 6 << 7
    e = struct.unpack_from("<Q", x, off_vdir + 8 * (ring6 + (30 >> 4)))[0]
    struct.pack_into("<Q", x, off_vdir + 8 * (ring6 + (30 >> 4)), e + (1 << 32))
    assert O.check_snapshot(bytes(x)).bad_vdir > 0
    # a consumed count off by one
    x = bytearray(b)
    v = struct.unpack_from("<I", x, off_vtk)[0]
    struct.pack_into("<I", x, off_vtk, v + 1)
    assert O.check_snapshot(bytes(x)).bad_vtaken > 0
    # the store loses a free segment id
    x = bytearray(b)
    n = struct.unpack_from("<I", x, off_vst + 256)[0]
    struct.pack_into("<I", x, off_vst + 256, n - 1)
    struct.pack_into("<Q", x, off_vst, (n - 1) + 0x80000000)
    struct.pack_into("<I", x, off_vss + 4 * (n - 1), 0xFFFFFFFF)
    assert O.check_snapshot(bytes(x)).bad_vstore > 0
    # a stray value in a slot no position holds
    x = bytearray(b)
    struct.pack_into("<I", x, off_sl + 4 * (63 * 16 + 3), 7)
    assert O.check_snapshot(bytes(x)).bad_ring_entry > 0
    # committed pages that do not match the classes' chunks
    assert O.check_snapshot(_va_state(lambda r, o, v: v.update(committed=[5]))).bad_committed > 0


# ---------------------------------------------------------------------------
# virtualised array chunk variant: segment count, sequential behaviour,
# snapshots
# ---------------------------------------------------------------------------

def _max_segments_touched(span, G, K):
    """Brute force: the most segments K queues of chunk ids can touch at
    once when they hold at most span entries together (a chunk is listed in
    at most one queue), over every split of the entries and every start
    offset of each queue inside its first segment."""
    f = [0] * (span + 1)   # most segments one queue of e entries touches
    for e in range(1, span + 1):
        f[e] = max(-(-(h + e) // G) - h // G for h in range(G))
    best = [0] * (span + 1)   # best[t]: most segments with t entries so far
    for _ in range(K):
        nxt = best[:]
        for t in range(span + 1):
            for e in range(1, span - t + 1):
                nxt[t + e] = max(nxt[t + e], best[t] + f[e])
        best = nxt
    return max(best)


def test_va_chunk_segments_closed_form():
    """M = ceil(span / 2^g) + 3K segments per shard, g = log2(span) - 3 in
    [4, 10]: the queues' storage (brute-forced above) plus one segment per
    queue on its way back to the store always fits."""
    for span, G, K in [(4, 16, 9), (40, 16, 3), (64, 16, 2), (33, 16, 4), (100, 32, 3)]:
        M = -(-span // G) + 3 * K
        assert _max_segments_touched(span, G, K) + K <= M, (span, G, K)
    for nbytes, C, shards in [(4 << 30, 8192, 0), (8 << 20, 8192, 1), (64 << 20, 16384, 4), (1 << 20, 4096, 0),
                              (64 * 8192, 8192, 64)]:
        N = nbytes // C
        S, L = O.shard_geometry(N, shards)
        g = min(10, max(4, L - 3))
        K = O.num_classes(C)
        assert O.va_chunk_log2_seg(nbytes, C, shards) == g
        assert O.va_chunk_segments(nbytes, C, shards) == -(-(1 << L) // (1 << g)) + 3 * K


@pytest.mark.parametrize("policy", [0, 1])
def test_va_chunk_allocator_behaves_as_the_chunk_variant(policy):
    """Storage in segments changes nothing a request sees: the same request
    stream gets the same offsets and NULLs as the chunk variant."""
    rng = np.random.default_rng(5)
    nbytes, C = 8 << 20, 8192
    a = O.OracleHeap(nbytes, C, O.VARIANT_CHUNK, policy=policy)
    b = O.OracleHeap(nbytes, C, O.VARIANT_VA_CHUNK, policy=policy)
    live = []
    for _ in range(6):
        sizes = inputs.sizes_log_uniform(3000, 4, 8192, int(rng.integers(1 << 30)))
        oa, ob = a.alloc_batch(sizes), b.alloc_batch(sizes)
        assert np.array_equal(oa, ob)
        live += [o for o in oa if o >= 0]
        rng.shuffle(live)
        half, live = live[: len(live) // 2], live[len(live) // 2:]
        fa = a.free_batch(np.array(half, dtype=np.int64))
        fb = b.free_batch(np.array(half, dtype=np.int64))
        assert np.array_equal(fa, fb)
    assert a.accounting() == b.accounting()


def _va_chunk_state(tamper=None):
    # one shard, 4 chunks of 4 KiB (K = 9, W = 4): chunk 0 class 6 with pages
    # 1 and 3 free (count 2), chunk 2 class 0 with page 5 free (count 1);
    # span 4 -> segments of 16 entries, M = 1 + 27, directory 4, store 32
    N, log2C, K = 4, 12, 9
    cls = [6, 0xFF, 0, 0xFF]
    cnt = [2, 0, 1, 0]
    bits = [[0] * 4 for _ in range(N)]
    bits[0][0] = (1 << 1) | (1 << 3)
    bits[2][0] = 1 << 5
    rings = {6: (0, 30, [0]), 0: (0, 15, [2])}
    va = dict(g=4, ldir=2, lstore=5, M=28, budget=0, committed=[0])
    if tamper:
        tamper(rings, cnt, va)
    return build_snapshot(N, log2C, 3, 2, cls, cnt, bits, [2], [0, 2, 1, 3], rings, va=va)


def test_va_chunk_snapshot_clean_and_planted_faults():
    rep = O.check_snapshot(_va_chunk_state())
    assert rep.ok_header and not rep.violations(), rep.violations()
    b = bytearray(_va_chunk_state())
    off_vdir, off_vtk, off_vst, off_vss = struct.unpack_from("<QQQQ", b, 136)
    # the class-6 queue (ring 6) at position 30: directory entry 30 >> 4 = 1
    x = bytearray(b)
    e = struct.unpack_from("<Q", x, off_vdir + 8 * ((6 << 2) + 1))[0]
    struct.pack_into("<Q", x, off_vdir + 8 * ((6 << 2) + 1), e ^ 1)
    assert O.check_snapshot(bytes(x)).violations()
    # a listed chunk whose count disagrees with its free bits
    assert O.check_snapshot(_va_chunk_state(lambda r, c, v: c.__setitem__(0, 3))).bad_count > 0
    # a chunk with free pages missing from its queue
    assert O.check_snapshot(_va_chunk_state(lambda r, c, v: r.update({0: (0, 15, [])}))).bad_ring_missing > 0
    # chunk queues keep the committed-page counter at zero
    assert O.check_snapshot(_va_chunk_state(lambda r, c, v: v.update(committed=[4]))).bad_committed > 0
    # the store loses a free segment id
    x = bytearray(b)
    n = struct.unpack_from("<I", x, off_vst + 256)[0]
    struct.pack_into("<I", x, off_vst + 256, n - 1)
    struct.pack_into("<Q", x, off_vst, (n - 1) + 0x80000000)
    struct.pack_into("<I", x, off_vss + 4 * (n - 1), 0xFFFFFFFF)
    assert O.check_snapshot(bytes(x)).bad_vstore > 0
    # a header whose segment count is not the closed form
    assert not O.check_snapshot(_va_chunk_state(lambda r, c, v: v.update(M=27))).ok_header


# ---------------------------------------------------------------------------
# virtualised list variants: sequential behaviour, snapshots
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("pair", [(O.VARIANT_VL_PAGE, O.VARIANT_VA_PAGE), (O.VARIANT_VL_CHUNK, O.VARIANT_CHUNK)])
def test_vl_allocator_behaves_as_its_array_counterpart(pair):
    """A list of segments instead of a directory changes nothing a request
    sees: vl-page answers as va-page (same shared page budget), vl-chunk as
    the chunk variant."""
    rng = np.random.default_rng(9)
    nbytes, C = 2 << 20, 8192
    a, b = O.OracleHeap(nbytes, C, pair[0]), O.OracleHeap(nbytes, C, pair[1])
    live = []
    for _ in range(6):
        sizes = inputs.sizes_log_uniform(1500, 4, 8192, int(rng.integers(1 << 30)))
        oa, ob = a.alloc_batch(sizes), b.alloc_batch(sizes)
        assert np.array_equal(oa, ob)
        live += [o for o in oa if o >= 0]
        rng.shuffle(live)
        half, live = live[: len(live) // 2], live[len(live) // 2:]
        assert np.array_equal(a.free_batch(np.array(half, dtype=np.int64)), b.free_batch(np.array(half, dtype=np.int64)))
    assert a.accounting() == b.accounting()


def _vl_state(variant, tamper=None):
    # one shard, 4 chunks of 4 KiB (K = 9, W = 4): chunk 0 class 6 with pages
    # 1 and 3 free, chunk 2 class 0 with page 5 free.  Page queues: the two
    # free pages of class 6 from position 30 (a chain of segments 1 and 2,
    # 16 entries each), one page of class 0 at position 15; chunk queues:
    # chunk 0 at position 31, chunk 2 at position 16 (head on a boundary)
    N, log2C, K = 4, 12, 9
    cls = [6, 0xFF, 0, 0xFF]
    cnt = [2, 0, 1, 0]
    bits = [[0] * 4 for _ in range(N)]
    bits[0][0] = (1 << 1) | (1 << 3)
    bits[2][0] = 1 << 5
    off = lambda c, k, p: ((c << log2C) + p * (16 << k)) >> 4
    if variant == O.VARIANT_VL_PAGE:
        rings = {6: (0, 31, [off(0, 6, 1), off(0, 6, 3)]), 0: (0, 15, [off(2, 0, 5)])}
        owned = {6: 1, 0: 1}
        va = dict(vl=True, g=4, ldir=0, lstore=6, M=64, budget=(64 - 27) << 4, committed=[4 + 256])
        log2q = 7
    else:
        rings = {6: (0, 31, [0]), 0: (0, 16, [2])}
        owned = {}
        va = dict(vl=True, g=4, ldir=0, lstore=5, M=28, budget=0, committed=[0])
        log2q = 2
    if tamper:
        tamper(rings, owned, va)
    return build_snapshot(N, log2C, variant, log2q, cls, cnt, bits, [2], [0, 2, 1, 3], rings, owned=owned, va=va)


@pytest.mark.parametrize("variant", [4, 5])
def test_vl_snapshot_clean_and_planted_faults(variant):
    rep = O.check_snapshot(_vl_state(variant))
    assert rep.ok_header and not rep.violations(), rep.violations()
    b = bytearray(_vl_state(variant))
    off_vdir, off_vtk, off_vst, off_vss = struct.unpack_from("<QQQQ", b, 136)
    off_cl = struct.unpack_from("<Q", b, 56)[0]
    M = struct.unpack_from("<I", b, 124)[0]
    # a broken link: the class-6 queue's first segment loses its successor
    # (page variant: its chain spans segments 1 and 2)
    x = bytearray(b)
    f = struct.unpack_from("<Q", x, off_cl + 512 * 6 + 392)[0]
    m0 = f & 0xFFFFFFFF
    struct.pack_into("<Q", x, off_vdir + 8 * (M + m0), (1 << 64) - 1)
    if variant == 4:
        assert O.check_snapshot(bytes(x)).bad_vdir > 0
    # a tag naming another queue
    x = bytearray(b)
    t = struct.unpack_from("<Q", x, off_vdir + 8 * m0)[0]
    struct.pack_into("<Q", x, off_vdir + 8 * m0, t + (1 << 32))
    assert O.check_snapshot(bytes(x)).bad_vdir > 0
    # a front word ahead of head
    x = bytearray(b)
    struct.pack_into("<Q", x, off_cl + 512 * 6 + 392, f + (1 << 32))
    assert O.check_snapshot(bytes(x)).violations()
    # a consumed count off by one
    x = bytearray(b)
    v = struct.unpack_from("<I", x, off_vtk + 4 * m0)[0]
    struct.pack_into("<I", x, off_vtk + 4 * m0, v + 1)
    assert O.check_snapshot(bytes(x)).bad_vtaken > 0
    # the store loses a free segment id
    x = bytearray(b)
    n = struct.unpack_from("<I", x, off_vst + 256)[0]
    struct.pack_into("<I", x, off_vst + 256, n - 1)
    struct.pack_into("<Q", x, off_vst, (n - 1) + 0x80000000)
    struct.pack_into("<I", x, off_vss + 4 * (n - 1), 0xFFFFFFFF)
    assert O.check_snapshot(bytes(x)).bad_vstore > 0
    # committed pages that do not match the classes' chunks
    assert O.check_snapshot(_vl_state(variant, lambda r, o, v: v.update(committed=[5]))).bad_committed > 0


# ---------------------------------------------------------------------------
# virtualised array page variant: the shared page budget, brute-forced
# ---------------------------------------------------------------------------
#
# A page queue in segments of G slots holds every segment from the one its
# head is in (slots before the head consumed, the segment not yet closed) to
# the one of its last entry; a segment whose last slot was consumed is on
# its way back to the store until its closer returns it.  A class that owns
# P pages has at most P entries queued.  The budget of a shard's classes
# must leave enough segments that a producer always finds one in the store
# (the reading of the paper's virtualised array: queues taking storage on
# demand), in every state where each queue's entries are contiguous and at
# most one segment per queue is being handed back.

def _held_segments(h, e, G):
    """Segments one queue holds, enumerated position by position: the head
    h slots into its segment, e entries from the head on."""
    return len({p // G for p in range(h + e)})


@functools.lru_cache(maxsize=None)
def _queue_worst(P, G):
    """Most segments one queue of a class owning P pages can need: every
    head offset, every entry count up to P, plus one being handed back."""
    if P == 0:
        return 0
    return max(_held_segments(h, e, G) for h in range(G) for e in range(P + 1)) + 1


def _most_segments(ppcs, G, budget):
    """Most segments the queues of one shard can need at once when its
    classes (pages per chunk ppcs) own at most `budget` pages together:
    over every split of the budget into whole chunks per class (group
    knapsack; each class's worst for a given chunk count from _queue_worst,
    or for large P or G from its closed form, checked against it below)."""
    best = [0] * (budget + 1)     # best[b]: most segments with b pages owned so far
    for ppc in ppcs:
        items = []
        last = None
        for c in range(1, budget // ppc + 1):
            P = c * ppc
            w = _queue_worst(P, G) if P <= 2 * G and G <= 16 else (P + 2 * G - 2) // G + 1
            if w != last:
                items.append((P, w))
                last = w
        nxt = best[:]
        for b in range(budget + 1):
            for P, w in items:
                if P > b:
                    break
                if best[b - P] + w > nxt[b]:
                    nxt[b] = best[b - P] + w
        best = nxt
    return max(best)


def test_queue_worst_closed_form_matches_the_enumeration():
    """The shortcut _most_segments takes for P > 2G (head one slot before its
    segment's end, P entries: ceil((G - 1 + P) / G) segments, plus the one
    handed back), checked against the enumeration where that is cheap."""
    for G in (4, 8, 16):
        for P in range(1, 6 * G):
            assert _queue_worst(P, G) == (P + 2 * G - 2) // G + 1, (G, P)


def test_va_budget_exhaustive_tiny():
    """Exhaustive over tiny shards: with a reserve of 3K segments (K queues)
    no split of the owned pages, no head offsets, entry counts or hand-backs
    need more than the shard's M segments; with a reserve of 2K, states
    that do exist in most of these shapes, so a budget that kept only 2K
    back would let a producer find the store empty."""
    import itertools
    short = []
    for K, G, ppcs in [(1, 4, (2,)), (2, 4, (4, 1)), (3, 4, (4, 2, 1)), (2, 8, (2, 1)), (3, 8, (8, 4, 1))]:
        for M in range(3 * K + 1, 3 * K + 4):
            worst = {}
            for reserve in (2, 3):
                budget = (M - reserve * K) * G
                most = 0
                ranges = [range(0, budget // p + 1) for p in ppcs]
                for chunks in itertools.product(*ranges):
                    P = [c * p for c, p in zip(chunks, ppcs)]
                    if sum(P) > budget:
                        continue
                    most = max(most, sum(_queue_worst(x, G) for x in P))
                worst[reserve] = most
                assert most == _most_segments(ppcs, G, budget), (K, G, ppcs, M, reserve)
            assert worst[3] <= M, (K, G, ppcs, M, worst)
            short.append(worst[2] > M)
    # a 2K reserve falls short wherever a class of few pages per chunk can
    # leave its queue two slots into a segment (not for every tiny shape)
    assert sum(short) >= len(short) // 2, short


@pytest.mark.parametrize("nbytes,C,S", [(1 << 20, 4096, 1), (1 << 20, 4096, 2), (2 << 20, 8192, 4),
                                        (4 << 20, 16384, 8), (512 << 10, 4096, 1)])
def test_va_budget_never_drains_the_store(nbytes, C, S):
    """The oracle's budget on real geometries (K classes of C / 16 / 2^k
    pages per chunk, the oracle's G and M): the worst state fits in the
    shard's M segments; a budget with a 2K reserve instead would not."""
    K = O.num_classes(C)
    G = 1 << O.va_log2_seg(nbytes, C, S)
    M = O.va_segments(nbytes, C, S)
    ppcs = [C // 16 >> k for k in range(K)]
    budget = O.va_budget(nbytes, C, S)
    assert 0 < budget
    assert _most_segments(ppcs, G, budget) <= M
    assert _most_segments(ppcs, G, (M - 2 * K) * G) > M
