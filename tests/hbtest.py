"""Helpers shared by the GPU tests: device buffers, pointer -> offset
conversion and the oracle-side checks applied to every GPU result."""
from __future__ import annotations

import sys

import numpy as np

import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_u64(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).to("cuda")


def dev_i64(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int64)).to("cuda")


def zeros_i64(n: int):
    import torch
    return torch.zeros(n, dtype=torch.int64, device="cuda")


def offsets(ptrs, base: int) -> np.ndarray:
    p = ptrs.cpu().numpy().view(np.uint64)
    return np.where(p == 0, -1, (p.astype(np.int64) - np.int64(base)))


def check_blocks(heap, sizes: np.ndarray, offs: np.ndarray, allow_null: bool = False):
    rep = O.check_blocks(heap.info.data_bytes, heap.info.chunk_bytes, sizes, offs)
    assert rep.n_bad_size_nonnull == 0, "non-NULL for an invalid size"
    assert rep.n_oob == 0 and rep.n_misaligned == 0 and rep.n_straddle == 0, (rep.n_oob, rep.n_misaligned)
    assert rep.n_overlap == 0, f"{rep.n_overlap} overlapping blocks"
    if not allow_null:
        assert rep.n_null_valid == 0, f"{rep.n_null_valid} NULL for valid requests"
    return rep


def check_snapshot(heap):
    snap = heap.snapshot()
    rep = O.check_snapshot(snap)
    assert rep.ok_header, "snapshot header"
    assert not rep.violations(), rep.violations()
    return snap, rep


def live_of(rep) -> list:
    return [int(x) for x in list(rep.live)[: rep.n_classes]]
