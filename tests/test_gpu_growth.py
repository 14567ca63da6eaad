"""GPU parity of the growth line: agents grow int32 lists by doubling
reallocation (dev_malloc / copy / dev_free inside persistent kernels), step
by step and as one replayed HIP graph.

Checked after every step against the oracle run through the same sequence
of allocations and frees: each list in bounds, aligned, in a class that
holds it, no two lists overlapping; per-class live counts equal to the
oracle's; every list holding exactly the words the oracle's pattern
function gives (sampled lists read back and compared on the host, all lists
checked on the device); no allocation failure; after releasing everything
and a trim, the heap state equals a fresh heap's byte for byte.
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


class OracleGrowth:
    """The same schedule through the sequential oracle: step 0 allocates
    16 B per agent; step s allocates twice the bytes for every agent with
    doublings >= s and then frees its old block."""

    def __init__(self, nbytes, chunk, variant, doublings):
        self.ref = O.OracleHeap(nbytes, chunk, variant)
        self.d = doublings
        self.bytes = np.zeros(len(doublings), dtype=np.uint64)
        self.offs = np.full(len(doublings), -1, dtype=np.int64)

    def step(self, s):
        if s == 0:
            self.bytes[:] = 16
            self.offs = self.ref.alloc_batch(self.bytes)
        else:
            act = np.nonzero(self.d >= s)[0]
            new_bytes = self.bytes[act] * 2
            new_offs = self.ref.alloc_batch(new_bytes)
            assert (new_offs >= 0).all()
            self.ref.free_batch(self.offs[act])
            self.offs[act] = new_offs
            self.bytes[act] = new_bytes

    def live(self):
        return self.ref.accounting()["live"]


def read_list(hb, ptr, nbytes):
    import torch
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    hb.hb_stream_copy(buf, int(ptr), nbytes)
    return buf.cpu().numpy().tobytes()


def check_state(hb, heap, gr, ref, seed, sample):
    ptrs, nbytes, fails = gr.export()
    assert fails == 0
    sizes = nbytes.cpu().numpy().view(np.uint64)
    assert (sizes == ref.bytes).all(), "list sizes differ from the schedule"
    offs = offsets(ptrs, heap.base)
    check_blocks(heap, sizes, offs)
    assert heap.pattern_check(ptrs, nbytes, seed) == 0
    p = ptrs.cpu().numpy().view(np.uint64)
    for a in sample:
        assert read_list(hb, p[a], int(sizes[a])) == O.pattern_bytes(seed, int(a), int(sizes[a])), f"agent {a}"
    snap, srep = check_snapshot(heap)
    assert live_of(srep) == ref.live()
    assert O.check_blocks_in_snapshot(snap, sizes, offs) == 0


@pytest.mark.parametrize("variant,width,chunk", [(0, 64, 8 * KiB), (1, 64, 8 * KiB), (0, 16, 16 * KiB),
                                                 (1, 1, 64 * KiB), (2, 64, 8 * KiB), (2, 32, 32 * KiB),
                                                 (3, 64, 8 * KiB), (3, 16, 32 * KiB), (4, 64, 8 * KiB),
                                                 (4, 32, 32 * KiB), (5, 64, 8 * KiB), (5, 16, 32 * KiB)])
def test_growth_steps_match_oracle(hb, variant, width, chunk):
    import torch
    nbytes, agents, steps, seed = 96 * MiB, 5000, 9, 0x51
    d = inputs.growth_doublings(agents, inputs.SEED_GROWTH)
    sample = np.random.default_rng(1).choice(agents, 40, replace=False)
    with hb.Heap(nbytes, chunk, variant=variant, width=width) as heap:
        fresh = heap.snapshot()
        with hb.Growth(heap, torch.from_numpy(d).to("cuda"), steps, seed) as gr:
            ref = OracleGrowth(nbytes, chunk, variant, d)
            for s in range(steps):
                say(f"case growth-steps variant={variant} width={width} chunk={chunk} step={s}")
                gr.step(s)
                ref.step(s)
                check_state(hb, heap, gr, ref, seed, sample)
            gr.release()
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


@pytest.mark.parametrize("variant", [0, 1])
def test_growth_graph_replays_match_eager(hb, variant):
    """The graph replays the same steps: every replay (with eager checks,
    releases and a trim between them) ends in the eager run's state."""
    import torch
    nbytes, chunk, agents, steps, seed = 64 * MiB, 8 * KiB, 3000, 9, 0x77
    d = inputs.growth_doublings(agents, inputs.SEED_GROWTH + 1)
    sample = np.arange(0, agents, 97)
    with hb.Heap(nbytes, chunk, variant=variant) as heap:
        fresh = heap.snapshot()
        with hb.Growth(heap, torch.from_numpy(d).to("cuda"), steps, seed) as gr:
            ref = OracleGrowth(nbytes, chunk, variant, d)
            for s in range(steps):
                gr.step(s)
                ref.step(s)
            check_state(hb, heap, gr, ref, seed, sample)
            _, eager_bytes, _ = gr.export()
            gr.release()
            for r in range(3):
                say(f"case growth-graph variant={variant} replay={r}")
                gr.run_graph()
                _, nb, fails = gr.export()
                assert fails == 0
                assert torch.equal(nb, eager_bytes)
                check_state(hb, heap, gr, ref, seed, sample)
                gr.release()
                if r == 1:
                    heap.trim()
                    assert heap.snapshot() == fresh
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
def test_growth_full_size(hb, variant):
    """2^18 agents on a 4 GiB heap, nine steps (16 B .. 4 KiB), checked after
    every step, then one graph replay checked again."""
    import torch
    w = inputs.GROWTH
    agents, steps, seed = w.threads, w.rounds, w.seed
    d = inputs.growth_doublings(agents, w.seed)
    sample = np.random.default_rng(2).choice(agents, 32, replace=False)
    with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant) as heap:
        fresh = heap.snapshot()
        with hb.Growth(heap, torch.from_numpy(d).to("cuda"), steps, seed) as gr:
            ref = OracleGrowth(w.heap_bytes, w.chunk_bytes, variant, d)
            for s in range(steps):
                say(f"case growth-full variant={variant} step={s}")
                gr.step(s)
                ref.step(s)
                check_state(hb, heap, gr, ref, seed, sample)
            gr.release()
            say(f"case growth-full variant={variant} graph")
            gr.run_graph()
            check_state(hb, heap, gr, ref, seed, sample)
            gr.release()
        heap.trim()
        assert heap.snapshot() == fresh
        assert heap.error() == 0


def test_growth_autotune_small(hb):
    import torch
    agents, steps = 4000, 9
    d = torch.from_numpy(inputs.growth_doublings(agents, inputs.SEED_GROWTH)).to("cuda")
    cands = [(c, v, w) for c in (8 * KiB, 32 * KiB) for v in (0, 1) for w in (16, 64)]
    cands.append((8 * KiB, 0, 64, hb.FLAG_EAGER))  # eager chunk retirement
    cands.append((8 * KiB, 1, 64, hb.FLAG_EAGER))  # eager with the page variant: not run
    cands.append((2 * KiB, 0, 64))  # invalid chunk size: must be reported as not run
    say("case growth-autotune")
    ms, best = hb.growth_autotune(64 * MiB, agents, d, steps, 3, cands, reps=3)
    assert ms[-1] < 0 and ms[-2] < 0 and ms[-3] > 0
    ran = [i for i, t in enumerate(ms) if t > 0]
    assert len(ran) == len(cands) - 2
    assert best == min(ran, key=lambda i: ms[i])


@pytest.mark.parametrize("variant", [0, 1])
def test_growth_ragged_last_wave_large_lists(hb, variant):
    """Every agent grows to 4 KiB and the last wave of the grid is partial:
    the wave-cooperative copies must cover every unit with fewer lanes."""
    import torch
    agents, steps, seed = 3 * 64 + 7, 9, 0x99
    d = np.full(agents, 8, dtype=np.int32)
    with hb.Heap(32 * MiB, 8 * KiB, variant=variant) as heap:
        with hb.Growth(heap, torch.from_numpy(d).to("cuda"), steps, seed) as gr:
            ref = OracleGrowth(32 * MiB, 8 * KiB, variant, d)
            for s in range(steps):
                say(f"case growth-ragged variant={variant} step={s}")
                gr.step(s)
                ref.step(s)
                check_state(hb, heap, gr, ref, seed, np.arange(agents - 10, agents))
            gr.release()
        assert heap.error() == 0
