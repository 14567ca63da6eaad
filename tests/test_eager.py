"""Eager chunk retirement (chunk variant): pins of the oracle's eager mode
and of the snapshot checker's eager layout.

The paper leaves open when a chunk whose pages are all free leaves its
size class (Results: chunks are split into pages of one class).  Eager
retirement returns it to its shard's pool at once.  Sequentially that is,
by definition, the lazy allocator with a trim after every free; the tests
below check the oracle's eager mode against exactly that, against capacity
closed forms (a heap refilled with another class after everything was freed
holds N * C / s pages of it, with no trim), and against small FIFO
sequences worked by hand.
"""
import struct

import numpy as np
import pytest

import oracle as O

KiB = 1024


@pytest.fixture(scope="module", autouse=True)
def _build():
    O.build(force=False)


# ---------------------------------------------------------------------------
# the sequential allocator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("C,shards,seed", [(4 * KiB, 1, 1), (8 * KiB, 1, 2), (8 * KiB, 2, 3), (4 * KiB, 4, 4)])
def test_eager_is_lazy_with_a_trim_after_every_free(C, shards, seed):
    """Catches: a retirement missed, done too early (a page still live), or
    leaving the chunk in its class's list."""
    rng = np.random.default_rng(seed)
    nbytes = 24 * C
    e = O.OracleHeap(nbytes, C, O.VARIANT_CHUNK, O.POLICY_LOWEST, shards, eager=True)
    z = O.OracleHeap(nbytes, C, O.VARIANT_CHUNK, O.POLICY_LOWEST, shards)
    live = []
    for step in range(3000):
        if live and rng.random() < 0.48:
            off = live.pop(int(rng.integers(len(live))))
            assert e.free(off) == z.free(off) == O.FREE_OK
            z.trim()
        else:
            n = int(rng.choice([16, 48, 200, 1000, C // 2, C]))
            a, b = e.alloc(n), z.alloc(n)
            assert a == b, (step, n)
            if a >= 0:
                live.append(a)
        if step % 97 == 0:
            assert e.accounting() == z.accounting(), step
    assert e.accounting() == z.accounting()


@pytest.mark.parametrize("C", [4 * KiB, 8 * KiB])
def test_eager_refill_with_another_class_holds_the_closed_form(C):
    """N * C / s pages of a class after every page of another was freed, with
    no trim; the lazy allocator keeps the chunks with the first class."""
    N = 32
    K = O.num_classes(C)
    for ka, kb in [(0, K - 1), (K - 1, 0), (3, 5), (2, 2)]:
        sa, sb = O.page_bytes(ka), O.page_bytes(kb)
        for eager in (True, False):
            h = O.OracleHeap(N * C, C, O.VARIANT_CHUNK, O.POLICY_FIFO, 1, eager=eager)
            offs = h.alloc_batch(np.full(N * C // sa + 3, sa, dtype=np.uint64))
            assert int((offs >= 0).sum()) == N * C // sa
            assert (h.free_batch(offs[offs >= 0]) == O.FREE_OK).all()
            got = int((h.alloc_batch(np.full(N * C // sb + 5, sb, dtype=np.uint64)) >= 0).sum())
            if eager or ka == kb:
                assert got == N * C // sb, (ka, kb, eager)
            else:
                assert got == 0, (ka, kb)
            # eager: the heap is full of the second class; lazy: the chunks
            # stay with the first (all their pages free) until a trim
            acct = h.accounting()
            assert acct["free_chunks"] == 0
            assert acct["chunks"][kb if got else ka] == N


def test_eager_fifo_pool_order_worked_by_hand():
    """One shard of 4 chunks of 4 KiB.  Whole-chunk blocks: chunks 0..3 in
    pool order; freeing chunk 2's block, then chunk 0's, puts them at the
    back of the pool in that order, so the next two allocations (of any
    class) get chunk 2, then chunk 0.  Catches: a retired chunk put at the
    front, or the pool rebuilt in ascending order (a trim's order)."""
    C = 4 * KiB
    h = O.OracleHeap(4 * C, C, O.VARIANT_CHUNK, O.POLICY_FIFO, 1, eager=True)
    assert [h.alloc(C) for _ in range(4)] == [0, C, 2 * C, 3 * C]
    assert h.alloc(16) == -1
    assert h.free(2 * C) == O.FREE_OK and h.free(0) == O.FREE_OK
    assert h.alloc(16) == 2 * C
    assert h.alloc(C) == 0
    assert h.alloc(C) == -1
    # chunk 2 serves 16 B pages 1, 2, ...: freeing page 0 lists nothing new
    assert h.alloc(16) == 2 * C + 16
    # the lazy allocator keeps chunks with their class until a trim
    z = O.OracleHeap(4 * C, C, O.VARIANT_CHUNK, O.POLICY_FIFO, 1)
    assert [z.alloc(C) for _ in range(4)] == [0, C, 2 * C, 3 * C]
    assert z.free(2 * C) == O.FREE_OK and z.free(0) == O.FREE_OK
    assert z.alloc(16) == -1
    z.trim()
    assert z.alloc(16) == 0


def test_eager_fifo_listed_chunk_leaves_its_queue():
    """A listed chunk made whole leaves its class queue: chunk 0 of the 2 KiB
    class (2 pages) gets both pages back; the queue's next chunk serves next.
    Worked by hand: chunks 0, 1 of 2 KiB pages; pages handed out 0:0, 0:1,
    1:0; frees of 0:1 (chunk 0 listed) and 0:0 (chunk 0 whole: retired).
    The queue then holds chunk 1 (page 1); the pool holds 2, 3, then 0."""
    C = 4 * KiB
    h = O.OracleHeap(4 * C, C, O.VARIANT_CHUNK, O.POLICY_FIFO, 1, eager=True)
    a = [h.alloc(2048) for _ in range(3)]
    assert a == [0, 2048, C]
    assert h.free(2048) == O.FREE_OK and h.free(0) == O.FREE_OK
    assert h.alloc(2048) == C + 2048          # chunk 1's free page, from the queue
    assert h.alloc(2048) == 2 * C             # queue empty: pool head, chunk 2
    assert [h.alloc(C) for _ in range(3)] == [3 * C, 0, -1]


def test_eager_mode_is_for_the_chunk_variant_of_a_fresh_heap():
    with pytest.raises(ValueError):
        O.OracleHeap(1 << 20, 8 * KiB, O.VARIANT_PAGE, eager=True)
    h = O.OracleHeap(1 << 20, 8 * KiB)
    h.alloc(16)
    assert O.lib().orc_set_eager(h.h) == -1


# ---------------------------------------------------------------------------
# the snapshot checker, eager layout
# ---------------------------------------------------------------------------

TOK_NONE, TOK_HELD = 0xFFFFFFFF, 0xFFFFFFFE
def STALE(k):
    """Count-word bit: the chunk has a stale entry in the queue of class k."""
    return 1 << (16 + k)


def tok(k, pos):
    return (k << 28) | (pos & 0x0FFFFFFF)


def build_eager(N, log2C, cls, bits, ct, pool, rings, log2_span=None, cnt32=None):
    """An eager-retirement snapshot of one shard: cls[c], bits[c] (list of W
    words), ct[c] = (token, count), pool = (head, entries) of the pool ring,
    rings[k] = (head, entries)."""
    K = log2C - 3
    W = (1 << log2C) // 1024
    if log2_span is None:
        log2_span = max(0, (N - 1).bit_length())
    span = 1 << log2_span
    log2q = log2_span + 1
    Q = 1 << log2q

    def al(x):
        return (x + 255) & ~255
    off_pool = 256
    off_cl = al(off_pool + 128)
    off_cls = al(off_cl + 512 * K)
    off_cnt = al(off_cls + N)
    off_bits = al(off_cnt + 4 * N)
    off_pid = al(off_bits + 8 * N * W)
    off_sl = al(off_pid + 4 * span)
    off_ct = al(off_sl + 4 * K * Q)
    total = al(off_ct + 8 * N)
    b = bytearray(total)
    struct.pack_into("<IIQIIIIIIIIQQQQQQQQ", b, 0, 0x48424850, 4, N << log2C, N, log2C, K, 0, W, log2q,
                     1, log2_span, off_pool, off_cl, off_cls, off_cnt, off_bits, off_pid, off_sl, total)
    struct.pack_into("<IIQ", b, 168, 1, 0, off_ct)
    phead, pents = pool
    struct.pack_into("<QIIII", b, off_pool, len(pents) + 0x80000000, N, 0, phead & 0xFFFFFFFF,
                     (phead + len(pents)) & 0xFFFFFFFF)
    for i in range(span):
        struct.pack_into("<I", b, off_pid + 4 * i, 0xFFFFFFFF)
    for q, e in enumerate(pents):
        struct.pack_into("<I", b, off_pid + 4 * ((phead + q) % span), e)
    b[off_cls:off_cls + N] = bytes(cls)
    for c in range(N):
        struct.pack_into("<I", b, off_cnt + 4 * c, (cnt32 or {}).get(c, 0))
        for w in range(W):
            struct.pack_into("<Q", b, off_bits + 8 * (w * N + c), bits[c][w])
        t, n = ct[c]
        struct.pack_into("<Q", b, off_ct + 8 * c, (t << 32) | n)
    for k in range(K):
        head, ents = rings.get(k, (0, []))
        struct.pack_into("<Q", b, off_cl + 512 * k, (len(ents) + 0x80000000) & 0xFFFFFFFF)
        struct.pack_into("<I", b, off_cl + 512 * k + 128, head & 0xFFFFFFFF)
        struct.pack_into("<I", b, off_cl + 512 * k + 256, (head + len(ents)) & 0xFFFFFFFF)
        for q in range(Q):
            struct.pack_into("<I", b, off_sl + 4 * (k * Q + q), 0xFFFFFFFF)
        for q, e in enumerate(ents):
            struct.pack_into("<I", b, off_sl + 4 * (k * Q + ((head + q) % Q)), e)
    return bytes(b)


def eager_state():
    """8 chunks of 4 KiB (K = 9; class 7 = 2 KiB pages, 2 per chunk; class
    0 = 16 B, 256 per chunk).  Chunk 0: class 7, page 1 free, listed at
    position 5 of its queue (head 4: position 4 holds a stale entry of
    chunk 6, whose count word carries the stale bit of class 7).  Chunk 1: class 7,
    both pages live (no token).  Chunk 2: class 0, 255 pages free, listed at
    position 0.  Chunks 3..7 unowned; the pool ring holds them from head 9
    in the order 5, 6, 3, 4, 7."""
    N, log2C = 8, 12
    full = (1 << 64) - 1
    cls = [7, 7, 0] + [0xFF] * 5
    bits = [[0] * 4 for _ in range(N)]
    bits[0][0] = 0b10
    bits[2] = [full - 1, full, full, full]
    ct = [(tok(7, 5), 1), (TOK_NONE, 0), (tok(0, 0), 255)] + [(TOK_NONE, 0)] * 5
    ct[6] = (TOK_NONE, STALE(7))
    pool = (9, [5, 6, 3, 4, 7])
    rings = {7: (4, [6, 0]), 0: (0, [2])}
    return N, log2C, cls, bits, ct, pool, rings


def check(*args, **kw):
    rep = O.check_snapshot(build_eager(*args, **kw))
    return rep


def test_eager_checker_accepts_a_consistent_state_and_counts_stale_entries():
    rep = check(*eager_state())
    assert rep.ok_header and rep.eager == 1
    assert rep.violations() == {}
    assert rep.stale_entries == 1
    assert rep.free_chunks == 5 and rep.live[7] == 3 and rep.live[0] == 1


def _planted(mut):
    N, log2C, cls, bits, ct, pool, rings = eager_state()
    cls, bits, ct = list(cls), [list(x) for x in bits], list(ct)
    rings = dict(rings)
    mut(cls, bits, ct, rings)
    return check(N, log2C, cls, bits, ct, pool, rings).violations()


def test_eager_checker_finds_planted_mistakes():
    # a whole chunk still listed is legal (a stale entry of its queue can
    # block its retirement), and reported
    N, log2C, cls, bits, ct, pool, rings = eager_state()
    bits = [list(x) for x in bits]
    bits[0][0] = 0b11
    ct = list(ct)
    ct[0] = (tok(7, 5), 2)
    rep = check(N, log2C, cls, bits, ct, pool, rings)
    assert rep.violations() == {} and rep.whole_owned == 1
    # a chunk with free pages whose token names no entry
    def moved(cls, bits, ct, rings):
        ct[0] = (tok(7, 6), 1)
    assert "bad_ring_missing" in _planted(moved)
    # an allocator's hold left behind
    def held(cls, bits, ct, rings):
        ct[0] = (TOK_HELD, 1)
    v = _planted(held)
    assert "bad_count" in v and "bad_ring_missing" in v
    # a chunk without free pages keeping a token
    def kept(cls, bits, ct, rings):
        ct[1] = (tok(7, 9), 0)
    assert "bad_count" in _planted(kept)
    # an unowned chunk with a token
    def freetok(cls, bits, ct, rings):
        ct[3] = (tok(0, 1), 0)
    assert "bad_free_chunk" in _planted(freetok)
    # a live entry whose count disagrees with the bits
    def miscount(cls, bits, ct, rings):
        ct[2] = (tok(0, 0), 254)
    assert "bad_count" in _planted(miscount)
    # a stale entry without the flag, or the flag without a stale entry
    def noflag(cls, bits, ct, rings):
        ct[6] = (TOK_NONE, 0)
    assert "bad_count" in _planted(noflag)
    def flagonly(cls, bits, ct, rings):
        ct[3] = (TOK_NONE, STALE(2))
    assert "bad_count" in _planted(flagonly)
    # the bit of another queue than the one holding the stale entry
    def otherqueue(cls, bits, ct, rings):
        ct[6] = (TOK_NONE, STALE(0))
    assert "bad_count" in _planted(otherqueue)
    # a bit beyond the classes
    def beyond(cls, bits, ct, rings):
        ct[6] = (TOK_NONE, STALE(7) | STALE(9))
    assert "bad_count" in _planted(beyond)
    # two stale entries of one chunk (the queue could overflow)
    def twostale(cls, bits, ct, rings):
        rings[7] = (3, [6, 6, 0])
        ct[0] = (tok(7, 5), 1)
    assert "bad_ring_dup" in _planted(twostale)
    # the flag does not count as free pages
    def flagged_live(cls, bits, ct, rings):
        ct[2] = (tok(0, 0), 255 | STALE(0))
        rings[0] = (0, [2])
    v = _planted(flagged_live)
    assert "bad_count" in v  # chunk 2 has no stale entry
    # the token names the entry but the chunk belongs to another class
    def wrongclass(cls, bits, ct, rings):
        rings[0] = (0, [0])
        ct[0] = (tok(0, 0), 1)
        rings[7] = (4, [6, 2])
    assert _planted(wrongclass)


def test_eager_checker_pool_ring():
    N, log2C, cls, bits, ct, pool, rings = eager_state()
    # an owned chunk in the pool
    assert "bad_pool" in check(N, log2C, cls, bits, ct, (9, [5, 6, 3, 4, 0]), rings).violations()
    # an unowned chunk missing from the pool
    assert "bad_pool" in check(N, log2C, cls, bits, ct, (9, [5, 6, 3, 4]), rings).violations()
    # the same chunk twice
    assert "bad_pool" in check(N, log2C, cls, bits, ct, (9, [5, 6, 3, 4, 7, 7]), rings).violations()
    # wrap-around of the ring positions is fine
    assert check(N, log2C, cls, bits, ct, ((1 << 32) - 2, [5, 6, 3, 4, 7]), rings).violations() == {}
    # the lazy count array must stay zero in eager mode
    v = check(N, log2C, cls, bits, ct, pool, rings, cnt32={0: 1}).violations()
    assert "bad_count" in v


class _BruteEager:
    """Eager retirement written out from its definition, in plain Python:
    chunks of C bytes, each unowned or owned by one class with a set of free
    pages; an allocation takes the lowest free page of the lowest chunk of
    its class that has one, else page 0 of the lowest unowned chunk; a free
    that leaves every page of its chunk free makes the chunk unowned."""

    def __init__(self, n_chunks, C):
        self.C, self.N = C, n_chunks
        self.cls = [None] * n_chunks
        self.free = [set() for _ in range(n_chunks)]

    def alloc(self, n):
        if n == 0 or n > self.C:
            return -1
        s = 16
        while s < n:
            s *= 2
        ppc = self.C // s
        for c in range(self.N):
            if self.cls[c] == s and self.free[c]:
                p = min(self.free[c])
                self.free[c].remove(p)
                return c * self.C + p * s
        for c in range(self.N):
            if self.cls[c] is None:
                self.cls[c] = s
                self.free[c] = set(range(1, ppc))
                return c * self.C
        return -1

    def free_(self, off):
        c, s = off // self.C, self.cls[off // self.C]
        self.free[c].add((off % self.C) // s)
        if len(self.free[c]) == self.C // s:
            self.cls[c], self.free[c] = None, set()


@pytest.mark.parametrize("C,seed", [(4 * KiB, 11), (8 * KiB, 12), (4 * KiB, 13)])
def test_eager_oracle_equals_brute_force(C, seed):
    """The oracle's eager mode (one shard, lowest-first) against the
    definition above, operation by operation, on random sequences that fill
    and drain a 12-chunk heap.  Catches: a retirement at the wrong count, a
    retired chunk not reusable by another class, the wrong chunk or page
    chosen after a retirement."""
    rng = np.random.default_rng(seed)
    N = 12
    o = O.OracleHeap(N * C, C, O.VARIANT_CHUNK, O.POLICY_LOWEST, 1, eager=True)
    b = _BruteEager(N, C)
    live = []
    for step in range(4000):
        if live and rng.random() < (0.3 if step % 800 < 400 else 0.7):
            off = live.pop(int(rng.integers(len(live))))
            assert o.free(off) == O.FREE_OK
            b.free_(off)
        else:
            n = int(rng.choice([1, 16, 17, 100, 512, 1000, C // 4, C // 2 + 1, C]))
            a, e = o.alloc(n), b.alloc(n)
            assert a == e, (step, n, a, e)
            if a >= 0:
                live.append(a)
    acct = o.accounting()
    assert acct["free_chunks"] == sum(c is None for c in b.cls)
