"""GPU parity of eager chunk retirement (chunk variant created with
HBHEAP_FLAG_EAGER): a chunk whose pages are all free again returns to its
shard's pool at once, while kernels run, instead of at the next trim.

Checked against the oracle's eager mode:

- a single device lane matches the FIFO oracle address for address;
- a heap filled with one class, emptied and refilled with another (no
  trim) holds exactly the closed-form capacity of the second, with every
  chunk retired exactly once (4, 8 and 64 KiB chunks);
- churn rounds keep the eager invariants (tokens, stale entries and their
  per-queue bits) and the oracle's live counts, across chunk sizes and
  aggregation widths;
- allocations and frees inside one kernel (the growth line) keep every
  list intact;
- frees into a retired or reused chunk are reported invalid and change
  nothing;
- at full size: the 4 GiB sweep with no trims gets each size's capacity,
  the 8 GiB churn matches the oracle's live counts;
- after a trim the state equals a fresh heap's byte for byte.
"""
import numpy as np
import pytest

import oracle as O
from paper_2504_18211_amd import inputs
from tests.hbtest import check_blocks, check_snapshot, dev_i64, dev_u64, live_of, offsets, say, zeros_i64

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18211_amd import hbheap
    hbheap.lib()
    O.build(force=False)
    return hbheap


def test_eager_needs_the_chunk_variant(hb):
    for v in (1, 2, 3, 4, 5):
        with pytest.raises(hb.HbHeapError) as e:
            hb.Heap(8 * MiB, 8 * KiB, variant=v, flags=hb.FLAG_EAGER)
        assert e.value.code == hb.E_INVAL
    with hb.Heap(8 * MiB, 8 * KiB, flags=hb.FLAG_EAGER) as heap:
        d = hb.heap_device_handle(heap.h)
        assert d.flags & hb.FLAG_EAGER and d.chunk_ct
        heap.set_flags(0)  # eager retirement stays: it is fixed at creation
        assert hb.heap_device_handle(heap.h).flags & hb.FLAG_EAGER
    with hb.Heap(8 * MiB, 8 * KiB) as heap:
        assert not hb.heap_device_handle(heap.h).chunk_ct


@pytest.mark.parametrize("seed,shards", [(1, 1), (2, 1), (3, 4), (4, 8)])
def test_eager_single_lane_replay_matches_fifo_oracle(hb, seed, shards):
    say(f"case eager-replay seed={seed} shards={shards}")
    nbytes, C = 32 * 8 * KiB, 8 * KiB
    ops = inputs.op_script(3000, seed, lo=1, hi=8 * KiB, p_free=0.45, p_invalid_size=0.05)
    ref_heap = O.OracleHeap(nbytes, C, 0, O.POLICY_FIFO, shards, eager=True)
    ref = ref_heap.replay(ops)
    with hb.Heap(nbytes, C, shards=shards, flags=hb.FLAG_EAGER) as heap:
        assert heap.info.n_shards == ref_heap.shards
        od, out = dev_i64(ops), zeros_i64(len(ops))
        heap.replay(od, out)
        got = out.cpu().numpy()
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"first mismatch at op {bad[:5]}: gpu {got[bad[:5]]} oracle {ref[bad[:5]]}"
        _, rep = check_snapshot(heap)
        a = ref_heap.accounting()
        assert rep.eager == 1
        assert live_of(rep) == a["live"]
        assert [int(x) for x in list(rep.chunks)[: rep.n_classes]] == a["chunks"]
        assert rep.free_chunks == a["free_chunks"]
        assert heap.error() == 0


@pytest.mark.parametrize("sa,sb,C", [(16, 8 * KiB, 8 * KiB), (8 * KiB, 16, 8 * KiB), (4 * KiB, 512, 8 * KiB),
                                     (100, 100, 8 * KiB), (16, 64 * KiB, 64 * KiB), (2 * KiB, 16, 4 * KiB)])
@pytest.mark.parametrize("shards", [1, 0])
@pytest.mark.parametrize("rows", [1, 4])
def test_eager_class_change_without_trim(hb, sa, sb, C, shards, rows):
    """16 MiB heap (2048 chunks of 8 KiB; 256 of 64 KiB, 4096 pages of 16 B
    each; 4096 of 4 KiB).  Class a fills it (exactly N * C / s_a succeed),
    every block is freed, and class b then gets exactly N * C / s_b -- no
    trim in between; each chunk was retired exactly once.  rows: requests
    per lane of the batch kernels."""
    nbytes = 16 * MiB
    N = nbytes // C
    with hb.Heap(nbytes, C, shards=shards, flags=hb.FLAG_EAGER | hb.FLAG_STATS, rows=rows) as heap:
        fresh = heap.snapshot()
        for rnd, s in enumerate((sa, sb)):
            cap = N * (C // O.page_bytes(O.class_of(s, C)))
            n = cap + 4096
            say(f"case eager-class-change sa={sa} sb={sb} C={C} shards={shards} rows={rows} phase={rnd} n={n}")
            sizes = np.full(n, s, dtype=np.uint64)
            sd, ptrs = dev_u64(sizes), zeros_i64(n)
            oom0 = heap.stats()["oom"]
            heap.alloc(sd, ptrs)
            offs = offsets(ptrs, heap.base)
            if int((offs >= 0).sum()) != cap:
                rep = O.check_snapshot(heap.snapshot())
                K = rep.n_classes
                assert False, dict(got=int((offs >= 0).sum()), cap=cap, err=heap.error(), stats=heap.stats(),
                                   bad=rep.violations(), free_chunks=rep.free_chunks, stale=rep.stale_entries,
                                   chunks=list(rep.chunks)[:K], free_pages=list(rep.free_pages)[:K])
            assert heap.stats()["oom"] - oom0 == n - cap
            check_blocks(heap, sizes, offs, allow_null=True)
            heap.pattern_write(ptrs, sd, 0xE1 + rnd)
            assert heap.pattern_check(ptrs, sd, 0xE1 + rnd) == 0
            _, rep = check_snapshot(heap)
            assert rep.free_chunks == 0
            st = zeros_i64(n).to(dtype=__import__("torch").int32)
            retired0 = heap.stats()["retired"]
            heap.free(ptrs, status=st)
            stn = st.cpu().numpy()
            assert (stn[offs >= 0] == hb.FREE_OK).all() and (stn[offs < 0] == hb.FREE_NULL).all()
            _, rep = check_snapshot(heap)
            assert rep.free_chunks == N and sum(rep.chunks[: rep.n_classes]) == 0
            assert heap.stats()["retired"] - retired0 == N
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


@pytest.mark.parametrize("shards,chunk,width", [(1, 8 * KiB, 64), (0, 8 * KiB, 64), (0, 64 * KiB, 64),
                                                (0, 4 * KiB, 16), (1, 16 * KiB, 1)])
@pytest.mark.parametrize("rows", [1, 4])
def test_eager_churn_rounds(hb, shards, chunk, width, rows):
    """256 MiB heap, 2^16 requests of log-uniform sizes in [4 B, 8 KiB] (about
    98 MB of pages live, mean class about 1490 B); each
    round frees a random half and allocates the freed slots with fresh sizes.
    Every round: blocks valid and non-overlapping, patterns intact, the
    snapshot consistent (eager invariants included), live counts equal to
    the oracle's.  At the end every block is freed: every chunk is back in
    the pools without a trim.  rows: requests per lane of the batch kernels
    (4 applies from width 16)."""
    import torch
    nbytes, C, n, rounds, seed = 256 * MiB, chunk, 1 << 16, 6, 0xE3
    N = nbytes // C
    ref = O.OracleHeap(nbytes, C, 0, O.POLICY_LOWEST, 1, eager=True)
    with hb.Heap(nbytes, C, shards=shards, flags=hb.FLAG_EAGER, width=width, rows=rows) as heap:
        fresh = heap.snapshot()
        sizes = inputs.sizes_log_uniform(n, 4, min(C, 8 * KiB), seed)
        sd, ptrs = dev_u64(sizes), zeros_i64(n)
        heap.alloc(sd, ptrs)
        roffs = ref.alloc_batch(sizes)
        assert (roffs >= 0).all()
        rng = np.random.default_rng(seed)
        for r in range(rounds):
            say(f"case eager-churn shards={shards} chunk={chunk} width={width} rows={rows} round={r}")
            offs = offsets(ptrs, heap.base)
            check_blocks(heap, sizes, offs)
            heap.pattern_write(ptrs, sd, seed + r)
            assert heap.pattern_check(ptrs, sd, seed + r) == 0
            snap, rep = check_snapshot(heap)
            assert live_of(rep) == ref.accounting()["live"]
            assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0
            idx = np.sort(rng.choice(n, n // 2, replace=False))
            ix = torch.from_numpy(idx).to("cuda")
            sub = ptrs[ix].contiguous()
            st = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
            heap.free(sub, status=st)
            assert (st.cpu().numpy() == hb.FREE_OK).all()
            assert (ref.free_batch(roffs[idx]) == O.FREE_OK).all()
            _, rep = check_snapshot(heap)
            assert live_of(rep) == ref.accounting()["live"]
            new = inputs.sizes_log_uniform(len(idx), 4, min(C, 8 * KiB), seed + 100 + r)
            sizes[idx] = new
            nd, nptr = dev_u64(new), zeros_i64(len(idx))
            heap.alloc(nd, nptr)
            ptrs[ix] = nptr
            sd = dev_u64(sizes)
            roffs[idx] = ref.alloc_batch(new)
            assert (roffs >= 0).all()
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        heap.free(ptrs, status=st)
        assert (st.cpu().numpy() == hb.FREE_OK).all()
        _, rep = check_snapshot(heap)
        # every chunk is back in the pools, except a whole one whose queue
        # still held a stale entry of it when it became whole (kept listed)
        assert sum(live_of(rep)) == 0
        assert rep.free_chunks + rep.whole_owned == N
        say(f"  chunks kept whole and listed: {rep.whole_owned}")
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


def test_eager_growth_in_one_kernel(hb):
    """Allocations and frees inside one persistent kernel (the growth line):
    chunks retire and change class while the kernel runs.  Lists intact,
    live counts equal to the oracle's, after a trim the fresh state."""
    import torch
    from tests.test_gpu_growth import OracleGrowth, check_state
    nbytes, chunk, agents, steps, seed = 96 * MiB, 8 * KiB, 5000, 9, 0x5E
    d = inputs.growth_doublings(agents, inputs.SEED_GROWTH)
    sample = np.random.default_rng(3).choice(agents, 40, replace=False)
    with hb.Heap(nbytes, chunk, flags=hb.FLAG_EAGER | hb.FLAG_STATS) as heap:
        fresh = heap.snapshot()
        with hb.Growth(heap, torch.from_numpy(d).to("cuda"), steps, seed) as gr:
            ref = OracleGrowth(nbytes, chunk, 0, d)
            for s in range(steps):
                say(f"case eager-growth step={s}")
                gr.step(s)
                ref.step(s)
                check_state(hb, heap, gr, ref, seed, sample)
            assert heap.stats()["retired"] > 0
            gr.release()
            say("case eager-growth graph")
            gr.run_graph()
            check_state(hb, heap, gr, ref, seed, sample)
            gr.release()
        _, rep = check_snapshot(heap)
        assert rep.free_chunks == nbytes // chunk
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


def test_eager_sweep_full_size(hb):
    """The measured sweep at full size -- 4 GiB heap, 8 KiB chunks, 2^20
    threads, 16 B .. 8 KiB -- on a chunk heap with eager retirement and no
    trim between sizes.  Each size gets exactly min(2^20, N * C / s)
    (8 KiB: half the requests fail): the chunks the previous size freed are
    back in the pools.  After every free launch no page is live and every
    chunk is in a pool (or kept whole behind a stale entry)."""
    w = inputs.SWEEP
    n, C = w.threads, w.chunk_bytes
    with hb.Heap(w.heap_bytes, C, flags=hb.FLAG_EAGER) as heap:
        N = heap.info.n_chunks
        fresh = heap.snapshot()
        ptrs = zeros_i64(n)
        for size in inputs.SWEEP_SIZES:
            k = O.class_of(size, C)
            cap = N * (C // O.page_bytes(k))
            sizes = inputs.sizes_fixed(n, size)
            sd = dev_u64(sizes)
            for it in range(2):
                say(f"case eager-sweep-full size={size} iteration={it}")
                heap.alloc(sd, ptrs)
                heap.pattern_write(ptrs, sd, w.seed)
                assert heap.pattern_check(ptrs, sd, w.seed) == 0
                offs = offsets(ptrs, heap.base)
                rep = check_blocks(heap, sizes, offs, allow_null=True)
                assert rep.n_nonnull == min(n, cap), (size, it, rep.n_nonnull, cap)
                if it == 0:
                    _, srep = check_snapshot(heap)
                    assert live_of(srep)[k] == min(n, cap)
                heap.free(ptrs)
            _, srep = check_snapshot(heap)
            assert sum(live_of(srep)) == 0
            assert srep.free_chunks + srep.whole_owned == N, (size, srep.free_chunks, srep.whole_owned)
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


def test_eager_churn_full_size(hb):
    """8 GiB heap, 2^21 requests of log-uniform sizes in [4 B, 8 KiB]; six
    rounds each free a random half and reallocate it with fresh sizes.  Every
    round: blocks valid and disjoint, patterns intact, snapshot consistent,
    live counts equal to the oracle's (eager mode)."""
    import torch
    w = inputs.CHURN
    n, seed, rounds = w.threads, w.seed, 6
    sizes = inputs.sizes_log_uniform(n, 4, 8 * KiB, seed)
    ref = O.OracleHeap(w.heap_bytes, w.chunk_bytes, 0, O.POLICY_LOWEST, 1, eager=True)
    roffs = ref.alloc_batch(sizes)
    assert (roffs >= 0).all()
    with hb.Heap(w.heap_bytes, w.chunk_bytes, flags=hb.FLAG_EAGER) as heap:
        N = heap.info.n_chunks
        fresh = heap.snapshot()
        sd, ptrs = dev_u64(sizes), zeros_i64(n)
        heap.alloc(sd, ptrs)
        rng = np.random.default_rng(seed)
        for r in range(rounds):
            say(f"case eager-churn-full round={r}")
            offs = offsets(ptrs, heap.base)
            check_blocks(heap, sizes, offs)
            heap.pattern_write(ptrs, sd, seed + r)
            assert heap.pattern_check(ptrs, sd, seed + r) == 0
            snap, rep = check_snapshot(heap)
            assert live_of(rep) == ref.accounting()["live"]
            idx = np.sort(rng.choice(n, n // 2, replace=False))
            ix = torch.from_numpy(idx).to("cuda")
            st = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
            heap.free(ptrs[ix].contiguous(), status=st)
            assert (st.cpu().numpy() == hb.FREE_OK).all()
            assert (ref.free_batch(roffs[idx]) == O.FREE_OK).all()
            new = inputs.sizes_log_uniform(len(idx), 4, 8 * KiB, seed + 1000 + r)
            sizes[idx] = new
            nptr = zeros_i64(len(idx))
            heap.alloc(dev_u64(new), nptr)
            ptrs[ix] = nptr
            sd = dev_u64(sizes)
            roffs[idx] = ref.alloc_batch(new)
            assert (roffs >= 0).all()
        st = torch.zeros(n, dtype=torch.int32, device="cuda")
        heap.free(ptrs, status=st)
        assert (st.cpu().numpy() == hb.FREE_OK).all()
        _, rep = check_snapshot(heap)
        assert sum(live_of(rep)) == 0 and rep.free_chunks + rep.whole_owned == N
        say(f"  chunks kept whole and listed: {rep.whole_owned}")
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


def test_eager_free_after_retirement_is_invalid(hb):
    """A block freed twice, the first free having made its chunk whole (so
    the chunk retired): the second free finds an unowned chunk and is
    reported invalid (status 2, the sticky invalid-free bit), and changes
    nothing -- the snapshot stays consistent and the chunk stays in its
    pool.  A free into a chunk reused by another class at an offset that is
    not a page of that class is invalid too."""
    import torch
    C = 8 * KiB
    with hb.Heap(1 * MiB, C, shards=1, flags=hb.FLAG_EAGER) as heap:
        N = heap.info.n_chunks
        sd, ptrs = dev_u64(np.full(4, 2 * KiB, dtype=np.uint64)), zeros_i64(4)
        heap.alloc(sd, ptrs)                 # one chunk, its four 2 KiB pages
        st = torch.zeros(4, dtype=torch.int32, device="cuda")
        heap.free(ptrs, status=st)
        assert (st.cpu().numpy() == hb.FREE_OK).all()
        _, rep = check_snapshot(heap)
        assert rep.free_chunks == N
        say("case eager-free-after-retirement")
        heap.free(ptrs, status=st)
        assert (st.cpu().numpy() == hb.FREE_INVALID).all()
        assert heap.error() & hb.ERR_INVALID_FREE
        _, rep = check_snapshot(heap)
        assert rep.free_chunks == N and sum(live_of(rep)) == 0
        hb.heap_clear_error(heap.h)
        # the chunk comes back as 3 KiB-class (4 KiB pages) blocks; an old
        # 2 KiB-page pointer at an odd page offset is not a page of it
        p4 = zeros_i64(N * 2)
        heap.alloc(dev_u64(np.full(N * 2, 4 * KiB, dtype=np.uint64)), p4)
        offs4 = offsets(p4, heap.base)
        assert (offs4 >= 0).all()
        old = offsets(ptrs, heap.base)
        odd = ptrs[torch.from_numpy(np.nonzero(old % (4 * KiB) != 0)[0]).to("cuda")].contiguous()
        st2 = torch.zeros(len(odd), dtype=torch.int32, device="cuda")
        heap.free(odd, status=st2)
        assert (st2.cpu().numpy() == hb.FREE_INVALID).all()
        _, rep = check_snapshot(heap)
        assert sum(live_of(rep)) == N * 2
        heap.free(p4)
        hb.heap_clear_error(heap.h)
        _, rep = check_snapshot(heap)
        assert rep.free_chunks == N
