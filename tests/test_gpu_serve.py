"""GPU parity of the serving line: batches of mixed allocations and frees,
admitted against the heap's free chunks, overlapped on K streams.

Each request's result is (status, class, checksum of the words read back).
The overlapped run, a run of the same requests one batch at a time, and the
oracle (the same requests through the sequential allocator, with the
checksum from the oracle's pattern) must agree exactly on every request.
At the end every live block is in bounds, aligned and non-overlapping, and
the per-class live counts equal the oracle's.
"""
import numpy as np
import pytest

import oracle as O
from paper_2504_18211_amd import inputs
from tests.hbtest import check_blocks, check_snapshot, live_of, offsets, say

pytestmark = pytest.mark.gpu

KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18211_amd import hbheap
    hbheap.lib()
    O.build(force=False)
    return hbheap


def oracle_serve(nbytes, chunk, variant, first, ops, seed):
    """Expected (status, class, checksum) per request, and the final live
    counts, from the sequential oracle."""
    ref = O.OracleHeap(nbytes, chunk, variant)
    R = len(ops)
    offs = np.full(R, -1, dtype=np.int64)
    status = np.zeros(R, dtype=np.uint8)
    for b in range(len(first) - 1):
        f0, f1 = int(first[b]), int(first[b + 1])
        seg = ops[f0:f1]
        ai = f0 + np.nonzero(seg >= 0)[0]
        fi = f0 + np.nonzero(seg < 0)[0]
        if len(ai):
            offs[ai] = ref.alloc_batch(ops[ai].astype(np.uint64))
            status[ai] = np.where(offs[ai] >= 0, 0, 4)
        if len(fi):
            tg = -ops[fi] - 1
            st = ref.free_batch(offs[tg])
            status[fi] = np.where(offs[tg] < 0, 3, st)
    is_alloc = ops >= 0
    tgt = np.where(is_alloc, np.arange(R), -ops - 1)
    size = np.where(is_alloc, ops, ops[tgt]).astype(np.uint64)
    ok_block = offs[tgt] >= 0
    cls = np.where(ok_block, O.classes(size, chunk), -1).astype(np.int8)
    sums = np.where(ok_block, O.pattern_sums(seed, tgt.astype(np.uint64), size), 0).astype(np.uint32)
    return status, cls, sums, ref.accounting()["live"], offs


def live_requests(ops):
    R = len(ops)
    freed = np.zeros(R, dtype=bool)
    freed[-ops[ops < 0] - 1] = True
    return np.nonzero((ops >= 0) & ~freed)[0]


def run_both(hb, nbytes, chunk, variant, plan, seed, slots, rate, admit=0.95, checks=True, flags=0):
    import torch
    out = {}
    for mode in ("mix", "alone"):
        with hb.Heap(nbytes, chunk, variant=variant, flags=flags) as heap:
            s = hb.serve_create(heap.h, slots, int(np.diff(plan.first).max()), len(plan.ops), admit, seed,
                                plan.free_lag)
            try:
                arr = inputs.arrivals_ns(len(plan.first) - 1, rate, seed) if mode == "mix" else None
                say(f"  run mode={mode} batches={len(plan.first) - 1} requests={len(plan.ops)}")
                r = hb.serve_run(s, plan.first, plan.ops, arr, alone=(mode == "alone"))
                assert heap.error() == 0
                if checks:
                    live = live_requests(plan.ops)
                    ptrs = torch.zeros(len(plan.ops), dtype=torch.int64, device="cuda")
                    hb.serve_export(s, 0, len(plan.ops), ptrs)
                    p = ptrs[torch.from_numpy(live).to("cuda")].contiguous()
                    sizes = plan.ops[live].astype(np.uint64)
                    offs = offsets(p, heap.base)
                    check_blocks(heap, sizes, offs)
                    _, srep = check_snapshot(heap)
                    r["live"] = live_of(srep)
                    r["chunks_in_use"] = hb.heap_chunks_in_use(heap.h)
                    assert r["chunks_in_use"] == heap.info.n_chunks - srep.free_chunks
            finally:
                hb.serve_destroy(s)
        out[mode] = r
    return out


def compare(out, exp):
    status, cls, sums, live, _ = exp
    for mode, r in out.items():
        assert (r["status"] == 0).all(), (mode, np.unique(r["status"], return_counts=True))
        assert np.array_equal(r["status"], status), mode
        assert np.array_equal(r["cls"], cls), mode
        assert np.array_equal(r["sum"], sums), mode
        if "live" in r:
            assert r["live"] == live, mode


@pytest.mark.parametrize("variant", [0, 1, 3, 5])
def test_serve_alone_equals_mix_equals_oracle(hb, variant):
    """Chunk, page, virtualised-array chunk and virtualised-list chunk heaps."""
    nbytes, chunk, seed = 256 * MiB, 8 * KiB, 0x5E
    plan = inputs.serve_plan(300, inputs.SEED_SERVE, warm_requests=60000, mean=512, lo=64, hi=4096)
    say(f"case serve-small variant={variant} warm_batches={plan.warm_batches}")
    out = run_both(hb, nbytes, chunk, variant, plan, seed, slots=4, rate=20000.0)
    compare(out, oracle_serve(nbytes, chunk, variant, plan.first, plan.ops, seed))
    st = out["mix"]["stats"]
    assert st["batches"] == 300 and st["peak_bound"] <= 0.95 * (nbytes // chunk)
    # the chunk usage came back with every batch's results
    assert st["monitor_reads"] == int((np.diff(plan.first) > 0).sum())
    assert (out["mix"]["latency_ns"] > 0).all()


def phase_change_plan(N, lag=2):
    """2 KiB blocks filling 45 % of N chunks, all freed, then 8 KiB blocks
    needing 45 % again."""
    n_small = int(0.45 * N) * 4             # 2 KiB pages, 4 per chunk
    per = 512
    small = [np.full(min(per, n_small - i), 2 * KiB, dtype=np.int64) for i in range(0, n_small, per)]
    R0 = sum(len(x) for x in small)
    frees = np.arange(R0, dtype=np.int64)
    free_batches = [-frees[i:i + per] - 1 for i in range(0, R0, per)]
    n_big = int(0.45 * N)
    big = [np.full(min(256, n_big - i), 8 * KiB, dtype=np.int64) for i in range(0, n_big, 256)]
    batches = small + [np.zeros(0, dtype=np.int64)] * lag + free_batches + big
    first = np.zeros(len(batches) + 1, dtype=np.uint64)
    first[1:] = np.cumsum([len(x) for x in batches])
    return inputs.ServePlan(first, np.concatenate(batches), len(small), lag), len(batches)


@pytest.mark.parametrize("variant", [0, 1])
def test_serve_admission_trims_between_phases(hb, variant):
    """2 KiB blocks fill 45 % of the chunks and are all freed; 8 KiB blocks
    then need 45 % again.  Chunks stay with their class until a trim, so the
    admission must stall, trim, and then admit; the results are unchanged."""
    nbytes, chunk, seed = 16 * MiB, 8 * KiB, 0x77
    N = nbytes // chunk
    n_small = int(0.45 * N) * 4             # 2 KiB pages, 4 per chunk
    per = 512
    small = [np.full(min(per, n_small - i), 2 * KiB, dtype=np.int64) for i in range(0, n_small, per)]
    R0 = sum(len(x) for x in small)
    lag = 2
    frees = np.arange(R0, dtype=np.int64)
    free_batches = [-frees[i:i + per] - 1 for i in range(0, R0, per)]
    n_big = int(0.45 * N)
    big = [np.full(min(256, n_big - i), 8 * KiB, dtype=np.int64) for i in range(0, n_big, 256)]
    # the first free batch trails the last small batch by `lag` batches
    batches = small + [np.zeros(0, dtype=np.int64)] * lag + free_batches + big
    first = np.zeros(len(batches) + 1, dtype=np.uint64)
    first[1:] = np.cumsum([len(x) for x in batches])
    ops = np.concatenate(batches)
    plan = inputs.ServePlan(first, ops, len(small), lag)
    say(f"case serve-trim variant={variant} batches={len(batches)}")
    out = run_both(hb, nbytes, chunk, variant, plan, seed, slots=4, rate=50000.0, admit=0.6)
    compare(out, oracle_serve(nbytes, chunk, variant, first, ops, seed))
    for mode in ("mix", "alone"):
        assert out[mode]["stats"]["trims"] >= 1, mode


def test_serve_eager_retirement_needs_no_trim(hb):
    """The same phase change on a chunk heap with eager retirement: the
    freed chunks are back in the pools as soon as their frees complete, so
    the admission never needs a trim; results equal the oracle's."""
    nbytes, chunk, seed = 16 * MiB, 8 * KiB, 0x78
    plan, nb = phase_change_plan(nbytes // chunk)
    say(f"case serve-eager batches={nb}")
    out = run_both(hb, nbytes, chunk, 0, plan, seed, slots=4, rate=50000.0, admit=0.6, flags=hb.FLAG_EAGER)
    compare(out, oracle_serve(nbytes, chunk, 0, plan.first, plan.ops, seed))
    for mode in ("mix", "alone"):
        assert out[mode]["stats"]["trims"] == 0, mode


def test_serve_page_class_capacity_is_not_admitted(hb):
    """Page variant on a small heap: 16 B pages of one class exceed the
    class's queue capacity long before the chunks run out.  The loop must
    refuse the batch (out of memory) rather than admit it and return NULLs."""
    nbytes, chunk = 16 * MiB, 8 * KiB
    with hb.Heap(nbytes, chunk, variant=hb.VARIANT_PAGE) as heap:
        S = heap.info.n_shards
        cap_pages = sum(min(nbytes // chunk // S, heap.info.ring_entries // 512) for _ in range(S)) * 512
        n = cap_pages + 4096
        per = 4096
        first = np.arange(0, n + per, per, dtype=np.uint64)
        first[-1] = n
        first = np.unique(first)
        ops = np.full(n, 16, dtype=np.int64)
        say(f"case serve-page-cap pages={cap_pages}")
        s = hb.serve_create(heap.h, 2, per, n, 0.95, 1, 1)
        try:
            for alone in (True, False):
                with pytest.raises(hb.HbHeapError) as e:
                    hb.serve_run(s, first, ops, inputs.arrivals_ns(len(first) - 1, 1e5, 1), alone=alone)
                assert e.value.code == hb.E_NOMEM
                heap.trim()
        finally:
            hb.serve_destroy(s)
        assert heap.error() == 0


@pytest.mark.parametrize("variant", [2, 4])
def test_serve_refuses_virtualised_page_heap(hb, variant):
    """The virtualised page variants share one page budget per shard, which
    the admission cannot bound: serve_create refuses them."""
    with hb.Heap(8 * MiB, 8 * KiB, variant=variant) as heap:
        with pytest.raises(hb.HbHeapError) as e:
            hb.serve_create(heap.h, 2, 64, 1000, 0.95, 1, 1)
        assert e.value.code == hb.E_INVAL


def test_serve_rejects_bad_plans(hb):
    with hb.Heap(8 * MiB, 8 * KiB) as heap:
        s = hb.serve_create(heap.h, 2, 64, 1000, 0.95, 1, 2)
        try:
            first = np.array([0, 4, 8, 12], dtype=np.uint64)
            good = np.array([16, 32, 64, 16, 100, 100, 100, 100, -1, -2, 16, 16], dtype=np.int64)
            for bad_ops in (
                np.where(np.arange(12) == 9, -1, good),       # request 0 freed twice
                np.where(np.arange(12) == 4, -2, good),       # free one batch after its allocation (lag 2)
                np.where(np.arange(12) == 8, -12, good),      # free of a later request
                np.where(np.arange(12) == 9, -9, good),       # free of a free
            ):
                with pytest.raises(hb.HbHeapError) as e:
                    hb.serve_run(s, first, bad_ops, alone=True)
                assert e.value.code == hb.E_INVAL
            with pytest.raises(hb.HbHeapError) as e:
                hb.serve_run(s, np.array([0, 65], dtype=np.uint64), np.full(65, 16, dtype=np.int64), alone=True)
            assert e.value.code == hb.E_INVAL                # batch above max_batch
            r = hb.serve_run(s, first, good, alone=True)
            assert (r["status"] == 0).all()
        finally:
            hb.serve_destroy(s)
    # a batch that cannot fit under the cap even on an empty heap
    with hb.Heap(8 * MiB, 8 * KiB) as heap:
        s = hb.serve_create(heap.h, 2, 1024, 1024, 0.5, 1, 1)
        try:
            with pytest.raises(hb.HbHeapError) as e:
                hb.serve_run(s, np.array([0, 1000], dtype=np.uint64), np.full(1000, 8 * KiB, dtype=np.int64),
                             alone=True)
            assert e.value.code == hb.E_NOMEM
        finally:
            hb.serve_destroy(s)


@pytest.mark.parametrize("variant", [1, 0])
def test_serve_full_size(hb, variant):
    """16 GiB heap, batches of mean 4096 requests (64 .. 65536), sizes
    log-uniform in [16 B, 8 KiB]: warm-up to about half the heap, then mixed
    allocations and frees; overlapped, alone and oracle results agree."""
    w = inputs.SERVE
    mean_block = 1817  # mean class size of log-uniform [16, 8192]
    warm = int(0.5 * w.heap_bytes / mean_block)
    plan = inputs.serve_plan(1400, w.seed, warm_requests=warm)
    say(f"case serve-full variant={variant} requests={len(plan.ops)} warm_batches={plan.warm_batches}")
    out = run_both(hb, w.heap_bytes, w.chunk_bytes, variant, plan, w.seed, slots=4, rate=5000.0)
    compare(out, oracle_serve(w.heap_bytes, w.chunk_bytes, variant, plan.first, plan.ops, w.seed))
