"""GPU parity: the HIP allocator (through the C ABI) against the CPU oracle.

Results of a concurrent allocator are not unique, so each GPU result is
checked against what the oracle fixes exactly: every block in bounds,
aligned to its class and inside one chunk; no two blocks overlap; every
block reads back its seeded pattern; per-class live counts equal the
oracle's for the same request stream; NULL only at the oracle's exact
capacity; the heap state is consistent at quiescence and byte-identical to a
fresh heap after everything is freed and trimmed.  A single device lane is
deterministic, and there the GPU must return the oracle's FIFO-policy
offsets one for one.
"""
import numpy as np
import pytest

import oracle as O
from paper_2504_18211_amd import inputs
from tests.hbtest import (check_blocks, check_snapshot, dev_i64, dev_u64, live_of, offsets, say,
                          zeros_i64)

pytestmark = pytest.mark.gpu

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30
# chunk, page, virtualised-array page and chunk, virtualised-list page and chunk
VARIANTS = [0, 1, 2, 3, 4, 5]


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18211_amd import hbheap
    hbheap.lib()
    O.build(force=False)
    return hbheap


def _oracle_cap(nbytes, C, variant, k, shards):
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


def _same_shards(heap, nbytes, C, requested):
    S, _ = O.shard_geometry(nbytes // C, requested)
    assert heap.info.n_shards == S, (heap.info.n_shards, S)
    return S


# ---------------------------------------------------------------------------
# tiny workload: 8 MiB heap, 8 KiB chunks, 1024 threads x 64 B, one round trip
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
def test_tiny_round_trip(hb, variant):
    w = inputs.TINY
    say(f"case tiny variant={variant}")
    sizes = inputs.sizes_fixed(w.threads, 64)
    with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant) as heap:
        fresh = heap.snapshot()
        assert not O.check_snapshot(fresh).violations()
        sd, ptrs = dev_u64(sizes), zeros_i64(w.threads)
        heap.alloc(sd, ptrs)
        heap.pattern_write(ptrs, sd, w.seed)
        assert heap.pattern_check(ptrs, sd, w.seed) == 0
        offs = offsets(ptrs, heap.base)
        check_blocks(heap, sizes, offs)
        snap, rep = check_snapshot(heap)
        ref = O.OracleHeap(w.heap_bytes, w.chunk_bytes, variant)
        ref.alloc_batch(sizes)
        assert live_of(rep) == ref.accounting()["live"]
        assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0
        # 1024 x 64 B = 8 chunks of 128 pages at least; bounded by one partial chunk per wave
        assert 8 <= sum(rep.chunks) <= 8 + 16
        st = zeros_i64(w.threads).to(dtype=__import__("torch").int32)
        heap.free(ptrs, status=st)
        assert (st.cpu().numpy() == 0).all()
        _, rep2 = check_snapshot(heap)
        assert sum(live_of(rep2)) == 0
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# single device lane: address-for-address parity with the FIFO oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("seed,shards", [(1, 1), (2, 1), (3, 4), (4, 8)])
def test_single_lane_replay_matches_fifo_oracle(hb, variant, seed, shards):
    say(f"case replay variant={variant} seed={seed} shards={shards}")
    nbytes, C = 32 * 8 * KiB, 8 * KiB
    ops = inputs.op_script(3000, seed, lo=1, hi=8 * KiB, p_free=0.4, p_invalid_size=0.05)
    ref = O.OracleHeap(nbytes, C, variant, O.POLICY_FIFO, shards).replay(ops)
    with hb.Heap(nbytes, C, variant=variant, shards=shards) as heap:
        _same_shards(heap, nbytes, C, shards)
        od, out = dev_i64(ops), zeros_i64(len(ops))
        heap.replay(od, out)
        got = out.cpu().numpy()
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"first mismatch at op {bad[:5]}: gpu {got[bad[:5]]} oracle {ref[bad[:5]]}"
        _, rep = check_snapshot(heap)
        acc_oracle = O.OracleHeap(nbytes, C, variant, O.POLICY_FIFO, shards)
        acc_oracle.replay(ops)
        a = acc_oracle.accounting()
        assert live_of(rep) == a["live"]
        assert [int(x) for x in list(rep.chunks)[: rep.n_classes]] == a["chunks"]
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# fixed-size sweep, reduced: 64 MiB heap (8192 chunks), 2^16 threads,
# 16 B .. 8 KiB; from 2 KiB up the heap runs out and exactly the oracle's
# capacity succeeds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shards", [1, 0])
@pytest.mark.parametrize("rows", [1, 4])
def test_sweep_small_exact_capacity(hb, variant, shards, rows):
    nbytes, C, n = 64 * MiB, 8 * KiB, 1 << 16
    with hb.Heap(nbytes, C, variant=variant, shards=shards, rows=rows) as heap:
        _same_shards(heap, nbytes, C, shards)
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        for size in inputs.SWEEP_SIZES:
            k = O.class_of(size, C)
            cap = _oracle_cap(nbytes, C, variant, k, shards)
            for it in range(2):
                say(f"case sweep-small variant={variant} shards={shards} rows={rows} size={size} iter={it}")
                sizes = inputs.sizes_fixed(n, size)
                sd = dev_u64(sizes)
                oom0 = heap.stats()["oom"]
                heap.alloc(sd, ptrs)
                heap.pattern_write(ptrs, sd, inputs.SEED_SWEEP)
                assert heap.pattern_check(ptrs, sd, inputs.SEED_SWEEP) == 0
                offs = offsets(ptrs, heap.base)
                rep = check_blocks(heap, sizes, offs, allow_null=True)
                assert rep.n_nonnull == min(n, cap), (rep.n_nonnull, cap)
                # requests answered NULL are counted (per home shard, summed)
                assert heap.stats()["oom"] - oom0 == n - min(n, cap)
                snap, srep = check_snapshot(heap)
                assert live_of(srep)[k] == min(n, cap)
                if n >= cap:
                    assert srep.free_pages[k] == 0
                    assert srep.free_chunks == 0 or variant not in (0, 3, 5)
                assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0
                heap.free(ptrs)
                _, srep = check_snapshot(heap)
                assert sum(live_of(srep)) == 0
            heap.trim()
            assert heap.snapshot() == fresh, f"not fresh after trim (size {size})"
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# stealing: 64 shards of one chunk each, far more requests than pages; every
# wave ends up taking from other shards and exactly the capacity succeeds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [0, 1, 3, 5])  # one-chunk shards leave segmented page variants no budget
def test_steal_exact_capacity(hb, variant):
    nbytes, C, n = 64 * 8 * KiB, 8 * KiB, 1 << 14
    with hb.Heap(nbytes, C, variant=variant, shards=64) as heap:
        _same_shards(heap, nbytes, C, 64)
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        for size in [16, 200, 1024, 8192]:
            say(f"case steal variant={variant} size={size}")
            k = O.class_of(size, C)
            cap = _oracle_cap(nbytes, C, variant, k, 64)
            sizes = inputs.sizes_fixed(n, size)
            sd = dev_u64(sizes)
            heap.alloc(sd, ptrs)
            offs = offsets(ptrs, heap.base)
            rep = check_blocks(heap, sizes, offs, allow_null=True)
            assert rep.n_nonnull == min(n, cap), (size, rep.n_nonnull, cap)
            heap.pattern_write(ptrs, sd, 9)
            assert heap.pattern_check(ptrs, sd, 9) == 0
            _, srep = check_snapshot(heap)
            if n >= cap:
                assert srep.free_pages[k] == 0
            heap.free(ptrs)
            heap.trim()
            assert heap.snapshot() == fresh
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# mixed-size churn, reduced: 2^16 threads, log-uniform 4 B .. 8 KiB, half
# freed and reallocated per round
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant,shards,flags", [(0, 1, 0), (0, 0, 0), (1, 1, 0), (1, 0, 0), (1, 0, 2), (2, 1, 0),
                                                  (2, 0, 0), (2, 0, 2), (3, 1, 0), (3, 0, 0), (4, 1, 0), (4, 0, 0),
                                                  (4, 0, 2), (5, 1, 0), (5, 0, 0), (0, 1, 8), (0, 0, 8)])
@pytest.mark.parametrize("rows", [1, 4])
def test_churn_small(hb, variant, shards, flags, rows):
    """flags 2: the page variant verifies every page it takes from a queue;
    flags 8: the chunk variant with eager retirement.  rows: requests per
    lane of the batch kernels."""
    import torch
    nbytes, C, n, rounds = 256 * MiB, 8 * KiB, 1 << 16, 4
    seed = inputs.SEED_CHURN
    sizes = inputs.sizes_log_uniform(n, 4, 8 * KiB, seed)
    ref = O.OracleHeap(nbytes, C, variant, eager=bool(flags & 8))
    ref_offs = ref.alloc_batch(sizes)
    with hb.Heap(nbytes, C, variant=variant, shards=shards, flags=flags, rows=rows) as heap:
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        heap.alloc(dev_u64(sizes), ptrs)
        for r in range(rounds + 1):
            say(f"case churn-small variant={variant} shards={shards} flags={flags} rows={rows} round={r}")
            if r:
                idx, new_sizes = inputs.churn_round(n, r, seed)
                idx_d = torch.from_numpy(idx).to("cuda")
                victims = ptrs[idx_d].contiguous()
                heap.free(victims)
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
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# free errors: double, invalid, NULL -- detected, ignored, state unharmed
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("rows", [1, 4])
def test_free_errors(hb, variant, rows):
    import torch
    say(f"case free-errors variant={variant} rows={rows}")
    nbytes, C = 1 * MiB, 8 * KiB
    with hb.Heap(nbytes, C, variant=variant, rows=rows) as heap:
        sizes = inputs.sizes_fixed(100, 64)
        ptrs = zeros_i64(100)
        heap.alloc(dev_u64(sizes), ptrs)
        p = ptrs.cpu().numpy()
        base = heap.base
        bad = np.array([p[0], p[0], p[1] + 16, base + nbytes + 64, 0, base + 100 * C, p[2], base - 64],
                       dtype=np.int64)
        st = torch.zeros(len(bad), dtype=torch.int32, device="cuda")
        heap.free(dev_i64(bad), status=st)
        s = st.cpu().numpy().tolist()
        assert sorted(s[:2]) == [0, 1]       # same page twice in one batch: one ok, one double
        assert s[2] == 2 and s[3] == 2 and s[4] == 3 and s[5] == 2 and s[6] == 0 and s[7] == 2
        err = heap.error()
        assert err & hb.ERR_DOUBLE_FREE and err & hb.ERR_INVALID_FREE and not err & hb.ERR_TIMEOUT
        _, srep = check_snapshot(heap)
        assert live_of(srep)[2] == 98
        st2 = torch.zeros(1, dtype=torch.int32, device="cuda")
        heap.free(dev_i64(np.array([p[0]])), status=st2)
        assert st2.item() == 1
        # sizes of the wrong class make a free invalid
        st3 = torch.zeros(1, dtype=torch.int32, device="cuda")
        heap.free(dev_i64(np.array([p[3]])), sizes=dev_u64(np.array([1000])), status=st3)
        assert st3.item() == 2
        stats = heap.stats()
        assert stats["double_free"] == 2 and stats["invalid_free"] == 5


# ---------------------------------------------------------------------------
# rows of consecutive pages: a ragged first batch makes the later rows start
# inside a bitmask word (and, from 1 KiB pages, cross chunks); the rows take
# their pages from the queue in order, free them, free them again (every
# request a double free, nothing changed), and take them back
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("size", [16, 1024, 8 * KiB])
def test_consecutive_rows_double_free(hb, variant, size):
    import torch
    say(f"case consecutive-rows variant={variant} size={size}")
    nbytes, C, n0, n = 64 * MiB, 8 * KiB, 37, 1 << 12
    k = O.class_of(size, C)
    with hb.Heap(nbytes, C, variant=variant, shards=1, rows=4) as heap:
        fresh = heap.snapshot()
        s0, s = inputs.sizes_fixed(n0, size), inputs.sizes_fixed(n, size)
        p0, p = zeros_i64(n0), zeros_i64(n)
        heap.alloc(dev_u64(s0), p0)
        sd = dev_u64(s)
        heap.alloc(sd, p)
        check_blocks(heap, s, offsets(p, heap.base))
        heap.free(p)                      # pages back to the queue in request order
        heap.alloc(sd, p)                 # rows of consecutive pages taken from the queue
        offs = offsets(p, heap.base)
        check_blocks(heap, s, offs)
        heap.pattern_write(p, sd, 0xC0)
        assert heap.pattern_check(p, sd, 0xC0) == 0
        _, rep = check_snapshot(heap)
        assert live_of(rep)[k] == n0 + n
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        heap.free(p, status=st)
        assert (st.cpu().numpy() == hb.FREE_OK).all()
        _, rep = check_snapshot(heap)
        assert live_of(rep)[k] == n0
        heap.free(p, status=st)           # the same rows again: every request a double free
        assert (st.cpu().numpy() == hb.FREE_DOUBLE).all()
        assert heap.error() & hb.ERR_DOUBLE_FREE
        assert heap.stats()["double_free"] == n
        _, rep = check_snapshot(heap)
        assert live_of(rep)[k] == n0
        heap.alloc(sd, p)
        check_blocks(heap, s, offsets(p, heap.base))
        _, rep = check_snapshot(heap)
        assert live_of(rep)[k] == n0 + n
        heap.free(p)
        heap.free(p0)
        heap.trim()
        assert heap.snapshot() == fresh


# ---------------------------------------------------------------------------
# payload harness on a partial last wave: large blocks are written and
# checked by the active lanes only, and must still be covered completely
# ---------------------------------------------------------------------------

def test_pattern_partial_wave_large_blocks(hb):
    import torch
    say("case pattern-partial-wave")
    n, size, seed = 64 + 6, 4 * KiB, 0x1234
    sizes = inputs.sizes_fixed(n, size)
    with hb.Heap(4 * MiB, 8 * KiB) as heap:
        sd, ptrs = dev_u64(sizes), zeros_i64(n)
        heap.alloc(sd, ptrs)
        heap.pattern_write(ptrs, sd, seed)
        assert heap.pattern_check(ptrs, sd, seed) == 0
        p = ptrs.cpu().numpy().view(np.uint64)
        for i in range(60, n):
            buf = torch.empty(size, dtype=torch.uint8, device="cuda")
            hb.hb_stream_copy(buf, int(p[i]), size)
            assert buf.cpu().numpy().tobytes() == O.pattern_bytes(seed, i, size), i
        heap.free(ptrs)


# ---------------------------------------------------------------------------
# aggregation width: 1, 16, 64 lanes per queue operation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("width", [1, 16, 64])
@pytest.mark.parametrize("rows", [1, 4])
def test_width_mixed_batch(hb, variant, width, rows):
    """rows 4 applies at widths 16 and 64 (a narrower width keeps one row)."""
    say(f"case width variant={variant} width={width} rows={rows}")
    nbytes, C, n = 64 * MiB, 16 * KiB, 20000  # ragged last wave
    sizes = inputs.sizes_log_uniform(n, 1, 16 * KiB, 77)
    sizes[::97] = 0
    sizes[5::101] = 16 * KiB + 1
    with hb.Heap(nbytes, C, variant=variant, width=width, rows=rows) as heap:
        fresh = heap.snapshot()
        sd, ptrs = dev_u64(sizes), zeros_i64(n)
        heap.alloc(sd, ptrs)
        offs = offsets(ptrs, heap.base)
        rep = check_blocks(heap, sizes, offs)
        assert rep.n_null == int((sizes == 0).sum() + (sizes > C).sum())
        heap.pattern_write(ptrs, sd, 5)
        assert heap.pattern_check(ptrs, sd, 5) == 0
        _, srep = check_snapshot(heap)
        ref = O.OracleHeap(nbytes, C, variant)
        ref.alloc_batch(sizes)
        assert live_of(srep) == ref.accounting()["live"]
        heap.free(ptrs)
        heap.trim()
        assert heap.snapshot() == fresh


# ---------------------------------------------------------------------------
# headline workload at full size: 4 GiB heap, 2^20 threads, 16 B .. 8 KiB
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant,rows", [(v, 0) for v in VARIANTS] + [(1, 1)])
def test_sweep_full_size(hb, variant, rows):
    """rows 0: the library's default (4 requests per lane); rows 1 on the
    page variant keeps one request per lane covered at full size too."""
    w = inputs.SWEEP
    n = w.threads
    with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant, rows=rows) as heap:
        _same_shards(heap, w.heap_bytes, w.chunk_bytes, 0)
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        for size in inputs.SWEEP_SIZES:
            say(f"case sweep-full variant={variant} rows={rows} size={size}")
            k = O.class_of(size, w.chunk_bytes)
            cap = _oracle_cap(w.heap_bytes, w.chunk_bytes, variant, k, 0)
            sizes = inputs.sizes_fixed(n, size)
            sd = dev_u64(sizes)
            for it in range(2):
                heap.alloc(sd, ptrs)
                heap.pattern_write(ptrs, sd, w.seed)
                assert heap.pattern_check(ptrs, sd, w.seed) == 0
                offs = offsets(ptrs, heap.base)
                rep = check_blocks(heap, sizes, offs, allow_null=True)
                assert rep.n_nonnull == min(n, cap), (size, rep.n_nonnull, cap)
                if it == 0:
                    snap, srep = check_snapshot(heap)
                    assert live_of(srep)[k] == min(n, cap)
                heap.free(ptrs)
            heap.trim()
            assert heap.snapshot() == fresh
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# mixed-size churn at full size: 8 GiB heap, 2^21 threads, log-uniform sizes
# in [4 B, 8 KiB], a random half freed and reallocated per round, 20 rounds
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
def test_churn_full_size(hb, variant):
    import torch
    w = inputs.CHURN
    n, seed = w.threads, w.seed
    sizes = inputs.sizes_log_uniform(n, 4, 8 * KiB, seed)
    ref = O.OracleHeap(w.heap_bytes, w.chunk_bytes, variant)
    ref_offs = ref.alloc_batch(sizes)
    with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant) as heap:
        _same_shards(heap, w.heap_bytes, w.chunk_bytes, 0)
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        heap.alloc(dev_u64(sizes), ptrs)
        for r in range(w.rounds + 1):
            say(f"case churn-full variant={variant} round={r}")
            if r:
                idx, new_sizes = inputs.churn_round(n, r, seed)
                idx_d = torch.from_numpy(idx).to("cuda")
                victims = ptrs[idx_d].contiguous()
                st = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
                heap.free(victims, status=st)
                assert int((st != 0).sum()) == 0
                ref.free_batch(ref_offs[idx])
                sizes[idx] = new_sizes
                fresh_ptrs = zeros_i64(len(idx))
                heap.alloc(dev_u64(new_sizes), fresh_ptrs)
                ptrs[idx_d] = fresh_ptrs
                ref_offs[idx] = ref.alloc_batch(new_sizes)
            sd = dev_u64(sizes)
            # blocks that survived earlier rounds are re-checked with the new ones
            heap.pattern_write(ptrs, sd, seed + r)
            assert heap.pattern_check(ptrs, sd, seed + r) == 0
            offs = offsets(ptrs, heap.base)
            check_blocks(heap, sizes, offs)
            if r % 10 == 0:
                snap, srep = check_snapshot(heap)
                assert live_of(srep) == ref.accounting()["live"]
                assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0
                say(f"  chunks in use {heap.info.n_chunks - srep.free_chunks} of {heap.info.n_chunks}")
        heap.free(ptrs)
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# the paper's own sweeps: 1024 allocations over the sizes, and 1 .. 2^20
# threads allocating 1000 B (4 GiB heap, 8 KiB chunks, two iterations each)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
def test_paper_sweeps(hb, variant):
    w = inputs.SWEEP
    points = [(inputs.PAPER_ALLOCS, s) for s in inputs.SWEEP_SIZES] + \
             [(t, inputs.PAPER_SIZE) for t in inputs.PAPER_THREADS]
    with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant) as heap:
        fresh = heap.snapshot()
        for n, size in points:
            say(f"case paper-sweep variant={variant} n={n} size={size}")
            sizes = inputs.sizes_fixed(n, size)
            sd, ptrs = dev_u64(sizes), zeros_i64(n)
            ref = O.OracleHeap(w.heap_bytes, w.chunk_bytes, variant)
            ref.alloc_batch(sizes)
            for it in range(2):
                heap.alloc(sd, ptrs)
                heap.pattern_write(ptrs, sd, it)
                assert heap.pattern_check(ptrs, sd, it) == 0
                offs = offsets(ptrs, heap.base)
                check_blocks(heap, sizes, offs)
                if it == 0 and n <= 4096:
                    _, srep = check_snapshot(heap)
                    assert live_of(srep) == ref.accounting()["live"]
                heap.free(ptrs)
            heap.trim()
            assert heap.snapshot() == fresh
        assert heap.error() == 0


# ---------------------------------------------------------------------------
# virtualised array page variant: the page budget of a shard matches the
# oracle's closed form, and one class can use all of it (more than the page
# variant's per-class queue allows)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [2, 4])
def test_va_budget_and_shared_capacity(hb, variant):
    nbytes, C = 2 * MiB, 8 * KiB
    with hb.Heap(nbytes, C, variant=variant, shards=1) as heap:
        assert heap.info.ring_entries == O.va_budget(nbytes, C, 1)
        fresh = heap.snapshot()
        n = 1 << 17
        for size in (16, 4096):
            say(f"case va-capacity size={size}")
            sizes = inputs.sizes_fixed(n, size)
            sd, ptrs = dev_u64(sizes), zeros_i64(n)
            heap.alloc(sd, ptrs)
            cap = _oracle_cap(nbytes, C, variant, O.class_of(size, C), 1)
            rep = check_blocks(heap, sizes, offsets(ptrs, heap.base), allow_null=True)
            assert rep.n_nonnull == min(n, cap)
            if size == 16:
                assert cap > _oracle_cap(nbytes, C, 1, 0, 1)
            heap.pattern_write(ptrs, sd, 3)
            assert heap.pattern_check(ptrs, sd, 3) == 0
            check_snapshot(heap)
            heap.free(ptrs)
            check_snapshot(heap)
            heap.trim()
            assert heap.snapshot() == fresh
        assert heap.error() == 0


def test_exhausted_class_beside_a_served_one(hb):
    """Page variant, one launch: every wave asks for 16 B pages far beyond
    that class's cap and for a few 4 KiB pages that fit.  Waves of a
    workgroup share out-of-memory proofs per class: the 16 B requests get
    exactly the cap, every 4 KiB request is served, and the NULLs counted
    equal the 16 B requests over the cap."""
    nbytes, C = 64 * MiB, 8 * KiB
    n = 1 << 18
    sizes = np.where(np.arange(n) % 32 == 31, 4096, 16).astype(np.uint64)
    cap16 = _oracle_cap(nbytes, C, 1, 0, 0)
    n16, n4k = int((sizes == 16).sum()), int((sizes == 4096).sum())
    ref = O.OracleHeap(nbytes, C, 1)
    roffs = ref.alloc_batch(sizes)
    assert int(((roffs >= 0) & (sizes == 16)).sum()) == cap16 < n16
    assert int(((roffs >= 0) & (sizes == 4096)).sum()) == n4k
    with hb.Heap(nbytes, C, variant=hb.VARIANT_PAGE) as heap:
        for it in range(2):
            say(f"case mixed-exhaustion iter={it}")
            sd, ptrs = dev_u64(sizes), zeros_i64(n)
            oom0 = heap.stats()["oom"]
            heap.alloc(sd, ptrs)
            offs = offsets(ptrs, heap.base)
            rep = check_blocks(heap, sizes, offs, allow_null=True)
            assert rep.n_nonnull == cap16 + n4k
            assert int(((offs >= 0) & (sizes == 4096)).sum()) == n4k
            assert int(((offs >= 0) & (sizes == 16)).sum()) == cap16
            assert heap.stats()["oom"] - oom0 == n16 - cap16
            heap.pattern_write(ptrs, sd, 11)
            assert heap.pattern_check(ptrs, sd, 11) == 0
            _, srep = check_snapshot(heap)
            assert live_of(srep)[0] == cap16 and live_of(srep)[8] == n4k
            heap.free(ptrs)
        heap.trim()
        assert heap.error() == 0
