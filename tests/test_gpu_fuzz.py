"""GPU schedule fuzzing: the allocator's concurrent protocol under widened
race windows.

The test build of the library (libhbheap_fuzz.so, HBHEAP_FUZZ=1) has fuzz
points between the atomic steps of reservations, takes, refills,
publications, frees, scans and segment hand-offs; with a seed set
(hb_fuzz_set), a wave sleeps at one point in four for a pseudo-random
number of s_sleep periods.  Interleavings that the normal timing makes rare
-- a refill overtaken between its pool take and its publication, a scan
between two of its reads, a segment closed while its neighbour installs --
then happen on small heaps with a few hundred waves.  Each case checks what
the oracle fixes regardless of the schedule: blocks valid and disjoint,
patterns read back, per-class live counts equal to the oracle's on the same
stream, NULL exactly at the oracle's capacity, consistent state at
quiescence, a fresh heap after free and trim, and no error bit.
"""
import numpy as np
import pytest

import oracle as O
from paper_2504_18211_amd import inputs
from tests.hbtest import check_blocks, check_snapshot, dev_u64, live_of, offsets, say, zeros_i64

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20
SEEDS = [0x5EED1, 0x5EED2, 0x5EED3, 0x5EED4, 0x5EED5, 0x5EED6]
MOST_SLEEPS = 32


def _set_fuzz(hbheap, seed, most):
    """hb_fuzz_set, with the HIP runtime's own error text on failure."""
    import ctypes as C
    rc = hbheap.lib().hb_fuzz_set(seed, most)
    if rc != hbheap.OK:
        hip = C.CDLL("libamdhip64.so")
        hip.hipGetErrorString.restype = C.c_char_p
        hip.hipGetErrorString.argtypes = [C.c_int]
        err = hip.hipGetLastError()
        raise AssertionError(f"hb_fuzz_set({seed:#x}, {most}) returned {rc}: HIP {err} {hip.hipGetErrorString(err)}")


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    from paper_2504_18211_amd import hbheap
    hbheap.lib()  # the normal library loads too (the other modules use it)
    hbheap.use_fuzz_library(True)
    try:
        hbheap.lib()
        yield hbheap
    finally:
        try:
            _set_fuzz(hbheap, 0, 0)
        finally:
            hbheap.use_fuzz_library(False)


def _cap(nbytes, C, variant, k, shards):
    """Pages of class k the heap holds: per shard min(chunks, cap) * ppc."""
    N = nbytes // C
    S, L = O.shard_geometry(N, shards)
    tot = 0
    for j in range(S):
        nj = min(N, (j + 1) << L) - (j << L)
        if variant in (0, 3, 5):
            cj = nj
        elif variant == 1:
            cj = min(nj, O.page_max_chunks(nbytes, C, k, S))
        else:
            cj = min(nj, O.va_budget(nbytes, C, S) // O.pages_per_chunk(C, k))
        tot += cj * O.pages_per_chunk(C, k)
    return tot


def test_fuzz_points_sleep(hb):
    """The fuzz points are live in this build: the same launch takes longer
    with sleeps on than off (a long sleep bound makes the gap plain)."""
    import torch
    n = 1 << 14
    sd = dev_u64(inputs.sizes_fixed(n, 64))
    ptrs = zeros_i64(n)

    def timed(seed, most):
        _set_fuzz(hb, seed, most)
        best = None
        with hb.Heap(8 * MiB, 8 * KiB, variant=1, shards=4) as heap:
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                heap.alloc(sd, ptrs)
                e1.record()
                torch.cuda.synchronize()
                heap.free(ptrs)
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) * 1e3
                best = us if best is None else min(best, us)
            assert heap.error() == 0
        return best

    off = timed(0, 0)
    on = timed(0x5EED1, 256)
    say(f"allocation launch: fuzz off {off:.1f} us, on {on:.1f} us")
    assert on > off + 20.0, (off, on)


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_fuzz_exact_capacity(hb, variant, seed):
    """2^16 requests on 4 shards over 1024 chunks; more requests than pages
    from 512 B up: exactly the capacity succeeds, twice in a row (refill,
    then reuse)."""
    _set_fuzz(hb, seed, MOST_SLEEPS)
    nbytes, C, n, shards = 8 * MiB, 8 * KiB, 1 << 16, 4
    with hb.Heap(nbytes, C, variant=variant, shards=shards) as heap:
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        for size in (16, 512, 4096, 8192):
            k = O.class_of(size, C)
            cap = _cap(nbytes, C, variant, k, shards)
            sizes = inputs.sizes_fixed(n, size)
            sd = dev_u64(sizes)
            for it in range(2):
                say(f"case fuzz-capacity variant={variant} seed={seed:#x} size={size} iter={it}")
                heap.alloc(sd, ptrs)
                heap.pattern_write(ptrs, sd, seed)
                assert heap.pattern_check(ptrs, sd, seed) == 0
                offs = offsets(ptrs, heap.base)
                rep = check_blocks(heap, sizes, offs, allow_null=True)
                assert rep.n_nonnull == min(n, cap), (size, it, rep.n_nonnull, cap)
                snap, srep = check_snapshot(heap)
                assert live_of(srep)[k] == min(n, cap)
                assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0
                heap.free(ptrs)
                _, srep = check_snapshot(heap)
                assert sum(live_of(srep)) == 0
            heap.trim()
            assert heap.snapshot() == fresh, f"not fresh after trim (size {size})"
        assert heap.error() == 0, hex(heap.error())


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("variant", [0, 1, 3, 5])  # one-chunk shards leave segmented page variants no budget
def test_fuzz_steal(hb, variant, seed):
    """64 one-chunk shards, 4096 requests: every wave takes from other
    shards (scan and steal), and exactly the capacity succeeds."""
    _set_fuzz(hb, seed, MOST_SLEEPS)
    nbytes, C, n = 64 * 8 * KiB, 8 * KiB, 1 << 12
    with hb.Heap(nbytes, C, variant=variant, shards=64) as heap:
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        for size in (16, 1024, 8192):
            say(f"case fuzz-steal variant={variant} seed={seed:#x} size={size}")
            k = O.class_of(size, C)
            cap = _cap(nbytes, C, variant, k, 64)
            sizes = inputs.sizes_fixed(n, size)
            sd = dev_u64(sizes)
            heap.alloc(sd, ptrs)
            offs = offsets(ptrs, heap.base)
            rep = check_blocks(heap, sizes, offs, allow_null=True)
            assert rep.n_nonnull == min(n, cap), (size, rep.n_nonnull, cap)
            heap.pattern_write(ptrs, sd, seed)
            assert heap.pattern_check(ptrs, sd, seed) == 0
            check_snapshot(heap)
            heap.free(ptrs)
            heap.trim()
            assert heap.snapshot() == fresh
        assert heap.error() == 0, hex(heap.error())


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("variant,flags", [(0, 0), (0, 8), (1, 0), (2, 0), (3, 0), (4, 0), (5, 0)])
def test_fuzz_churn(hb, variant, flags, seed):
    """2^15 requests of mixed sizes (log-uniform 4 B .. 8 KiB) on a 64 MiB
    heap of 4 shards, half freed and reallocated per round (frees and
    refills of many classes interleave); flags 8: the chunk variant with
    eager retirement."""
    import torch
    _set_fuzz(hb, seed, MOST_SLEEPS)
    nbytes, C, n, rounds = 64 * MiB, 8 * KiB, 1 << 15, 3
    sizes = inputs.sizes_log_uniform(n, 4, 8 * KiB, seed)
    ref = O.OracleHeap(nbytes, C, variant, shards=4, eager=bool(flags & 8))
    ref_offs = ref.alloc_batch(sizes)
    assert (ref_offs >= 0).all()  # the stream fits: every request is served
    with hb.Heap(nbytes, C, variant=variant, flags=flags, shards=4) as heap:
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        heap.alloc(dev_u64(sizes), ptrs)
        for r in range(rounds + 1):
            say(f"case fuzz-churn variant={variant} flags={flags} seed={seed:#x} round={r}")
            if r:
                idx, new_sizes = inputs.churn_round(n, r, seed)
                idx_d = torch.from_numpy(idx).to("cuda")
                heap.free(ptrs[idx_d].contiguous())
                ref.free_batch(ref_offs[idx])
                sizes[idx] = new_sizes
                fresh_ptrs = zeros_i64(len(idx))
                heap.alloc(dev_u64(new_sizes), fresh_ptrs)
                ptrs[idx_d] = fresh_ptrs
                ref_offs[idx] = ref.alloc_batch(new_sizes)
            sd = dev_u64(sizes)
            heap.pattern_write(ptrs, sd, seed)
            assert heap.pattern_check(ptrs, sd, seed) == 0
            offs = offsets(ptrs, heap.base)
            check_blocks(heap, sizes, offs)
            snap, srep = check_snapshot(heap)
            assert live_of(srep) == ref.accounting()["live"]
            assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0
        heap.free(ptrs)
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0, hex(heap.error())
