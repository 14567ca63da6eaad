"""GPU: heap_chunks_in_use_noalloc -- the entry point for callers that cannot
allocate (its staging is a fixed device array of the library, not memory
allocated per call) -- against heap_chunks_in_use, through the C ABI, on
two calls in a row, the second on a smaller heap (fewer chunks, fewer
classes), so that the shared staging holds the first call's words when the
second one runs."""
import ctypes as C

import numpy as np
import pytest

from tests.hbtest import dev_u64, say, zeros_i64

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20


@pytest.fixture(scope="module")
def hb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_18211_amd import hbheap
    hbheap.lib()
    return hbheap


def _count_both(hb, heap):
    import torch
    want = hb.heap_chunks_in_use(heap.h)
    out = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    L = hb.lib()
    rc = L.heap_chunks_in_use_noalloc(C.c_void_p(heap.h), C.c_void_p(out.data_ptr()),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == hb.OK
    torch.cuda.synchronize()
    return want, int(out.item())


def test_noalloc_matches_chunks_in_use(hb):
    # first call: 64 MiB heap of 8 KiB chunks (8192 chunks, 10 classes),
    # page variant, 20000 blocks of mixed sizes
    say("case noalloc 64 MiB page variant")
    with hb.Heap(64 * MiB, 8 * KiB, variant=hb.VARIANT_PAGE) as a:
        rng = np.random.default_rng(7)
        sizes = rng.integers(1, 8 * KiB, size=20000, dtype=np.uint64)
        ptrs = zeros_i64(len(sizes))
        a.alloc(dev_u64(sizes), ptrs)
        want, got = _count_both(hb, a)
        assert got == want and want > 0, (got, want)
        a.free(ptrs)
        a.trim()
        want0, got0 = _count_both(hb, a)
        assert got0 == want0 == 0
        a.alloc(dev_u64(sizes), ptrs)
        want1, got1 = _count_both(hb, a)
        assert got1 == want1 == want
    # second call: a smaller heap (8 MiB of 4 KiB chunks: 2048 chunks, 9
    # classes), chunk variant, 300 blocks of 4 KiB (one chunk each)
    say("case noalloc 8 MiB chunk variant")
    with hb.Heap(8 * MiB, 4 * KiB, variant=hb.VARIANT_CHUNK) as b:
        sizes = np.full(300, 4 * KiB, dtype=np.uint64)
        ptrs = zeros_i64(len(sizes))
        b.alloc(dev_u64(sizes), ptrs)
        want, got = _count_both(hb, b)
        assert got == want == 300, (got, want)


def test_noalloc_rejects_null(hb):
    import torch
    L = hb.lib()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert L.heap_chunks_in_use_noalloc(None, C.c_void_p(out.data_ptr()), None) == hb.E_INVAL
    with hb.Heap(8 * MiB, 8 * KiB) as h:
        assert L.heap_chunks_in_use_noalloc(C.c_void_p(h.h), None, None) == hb.E_INVAL
