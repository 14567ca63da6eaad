"""GPU: the bounded-wait path.  Every wait of the allocator (a slot whose
producer is late, a store or pool that is momentarily empty, an exhaustion
proof that sees holds in flight) gives up after the heap's spin_cap
iterations, sets HBHEAP_ERR_TIMEOUT in the sticky error word and answers the
request NULL, so that no kernel can hang on a heap that cannot make progress.
The paper reports timeouts and deadlocks of the ported allocator (Results);
this is the answer the library gives to them, tested through the C ABI.

The forced case makes a wait certain without touching the GPU's control
flow: at quiescence, the host overwrites a published queue slot with the
empty mark (the state word still counts the entry), so the next taker of
that position waits for a producer that never comes; with spin_cap = 1 it
gives up after one backoff.  The contended case only bounds what may
happen: with spin_cap = 1 a heavily oversubscribed heap may or may not time
out, but every launch returns, every block handed out is valid and no two
overlap, and the only error bit that may be set is the timeout.
"""
import numpy as np
import pytest

from tests.hbtest import check_blocks, dev_u64, offsets, say, zeros_i64

pytestmark = pytest.mark.gpu

MiB = 1 << 20
EMPTY = 0xFFFFFFFF


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18211_amd import hbheap
    hbheap.lib()
    return hbheap


def _plant_empty(hb, heap):
    """Overwrite ring positions 0..3 of queue (shard 0, class 0) with the
    empty mark, through the library's 16-byte copy kernel."""
    import torch
    d = hb.heap_device_handle(heap.h)
    assert d.n_shards == 1 and d.slots % 16 == 0 and d.log2q >= 2
    src = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    hb.hb_stream_copy(int(d.slots), src, 16)
    torch.cuda.synchronize()


@pytest.mark.parametrize("variant", [0, 1])
def test_forced_timeout(hb, variant):
    """A published slot emptied behind the queue's back: the taker of its
    position gives up after spin_cap backoffs, the timeout bit is set and
    counted, the launch returns, and the heap can still be destroyed."""
    import torch
    say(f"case forced timeout variant={variant}")
    heap = hb.Heap(8 * MiB, 8192, variant=variant, spin_cap=1, shards=1)
    try:
        one = dev_u64(np.array([16], dtype=np.uint64))
        p0 = zeros_i64(1)
        heap.alloc(one, p0)
        torch.cuda.synchronize()
        assert int(p0.item()) != 0 and heap.error() == 0
        # the refill published the rest of the chunk (page variant: its free
        # pages from position 0; chunk variant: the chunk itself at 0)
        _plant_empty(hb, heap)
        p1 = zeros_i64(1)
        heap.alloc(one, p1)
        torch.cuda.synchronize()
        err = heap.error()
        assert err == hb.ERR_TIMEOUT, hex(err)
        assert heap.stats()["timeouts"] >= 1
        if variant == 1:
            # the page variant answers the position it could not read NULL
            assert int(p1.item()) == 0
        else:
            # the chunk variant moves on to a fresh chunk of the pool
            assert int(p1.item()) not in (0, int(p0.item()))
    finally:
        heap.close()


@pytest.mark.parametrize("variant", [0, 1])
def test_contended_small_spin_cap(hb, variant):
    """2^16 lanes ask for 8 KiB pages of a 1024-chunk heap (64 times more
    than it holds) and then free them, with spin_cap = 1: every launch
    returns, the blocks handed out are valid and disjoint, and at most the
    timeout bit is set."""
    import torch
    say(f"case contended spin_cap=1 variant={variant}")
    n = 1 << 16
    sizes = np.full(n, 8192, dtype=np.uint64)
    with hb.Heap(8 * MiB, 8192, variant=variant, spin_cap=1) as heap:
        sd, ptrs = dev_u64(sizes), zeros_i64(n)
        heap.alloc(sd, ptrs)
        torch.cuda.synchronize()
        offs = offsets(ptrs, heap.base)
        rep = check_blocks(heap, sizes, offs, allow_null=True)
        ok = int((offs >= 0).sum())
        assert 0 < ok <= heap.info.n_chunks
        say(f"  served {ok} of {n}, error word {heap.error():#x}, timeouts {heap.stats()['timeouts']}")
        heap.free(ptrs)
        torch.cuda.synchronize()
        assert heap.error() & ~hb.ERR_TIMEOUT == 0, hex(heap.error())
        del rep
