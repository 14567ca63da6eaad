"""Seeded synthetic workloads shared by the device path's tests, the oracle's
tests and the benchmark.

This module only draws numbers: request sizes, which blocks to free, growth
schedules, arrival processes.  It holds none of the allocator's arithmetic
(no size classes, no geometry), so both sides of a parity test can be fed
from it without sharing the method's code.

The shapes follow the paper's driver (Methods: many threads allocate in
parallel, write data, read it back and free, ten times over) and the
workloads this library is measured on:

* ``tiny``   -- 8 MiB heap, 8 KiB chunks, 1024 threads x 64 B, one round;
* ``sweep``  -- 4 GiB heap, 2^20 threads, one fixed size per launch swept over
  powers of two 16 B .. 8 KiB, 10 iterations per size;
* ``churn``  -- 8 GiB heap, 2^21 threads, log-uniform sizes in [4 B, 8 KiB],
  50 % freed and reallocated per round, 20 rounds;
* ``growth`` -- 2^18 agents doubling an int32 list 16 B -> 4 KiB over 9 steps
  with geometric per-agent growth;
* ``serve``  -- Poisson batches (mean 4096 requests, 64..65536) of mixed
  allocations and frees, sizes log-uniform in [16 B, 8 KiB], 16 GiB heap.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

KiB = 1 << 10
MiB = 1 << 20
GiB = 1 << 30

SEED_TINY = 0xC0F1
SEED_SWEEP = 0xC0F2
SEED_CHURN = 0xC0F3
SEED_GROWTH = 0xC0F4
SEED_SERVE = 0xC0F5

SWEEP_SIZES = [16 << i for i in range(10)]  # 16 B .. 8 KiB

# the paper's own driver sweeps (Results): 1024 allocations over a range of
# sizes, and a range of thread counts allocating 1000 B each
PAPER_ALLOCS = 1024
PAPER_SIZE = 1000
PAPER_THREADS = [1 << (2 * i) for i in range(11)]  # 1 .. 2^20


@dataclass(frozen=True)
class Workload:
    name: str
    heap_bytes: int
    chunk_bytes: int
    threads: int
    seed: int
    rounds: int


TINY = Workload("tiny", 8 * MiB, 8 * KiB, 1024, SEED_TINY, 1)
SWEEP = Workload("sweep", 4 * GiB, 8 * KiB, 1 << 20, SEED_SWEEP, 10)
CHURN = Workload("churn", 8 * GiB, 8 * KiB, 1 << 21, SEED_CHURN, 20)
GROWTH = Workload("growth", 4 * GiB, 8 * KiB, 1 << 18, SEED_GROWTH, 9)
SERVE = Workload("serve", 16 * GiB, 8 * KiB, 4096, SEED_SERVE, 0)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sizes_fixed(n: int, size: int) -> np.ndarray:
    return np.full(n, size, dtype=np.uint64)


def sizes_log_uniform(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """u ~ U[ln lo, ln(hi+1)), size = min(hi, floor(e^u))."""
    u = rng(seed).uniform(math.log(lo), math.log(hi + 1), size=n)
    s = np.floor(np.exp(u)).astype(np.uint64)
    return np.minimum(s, np.uint64(hi))


def churn_round(n: int, round_idx: int, seed: int, lo: int = 4, hi: int = 8 * KiB):
    """Indices freed in round ``round_idx`` (a random half) and their new sizes."""
    g = rng(seed + 1 + round_idx)
    idx = np.sort(g.permutation(n)[: n // 2]).astype(np.int64)
    new_sizes = sizes_log_uniform(idx.shape[0], lo, hi, seed + 1000 + round_idx)
    return idx, new_sizes


def growth_doublings(agents: int, seed: int, p: float = 0.3, cap: int = 8) -> np.ndarray:
    """Per-agent number of doublings: min(cap, G) with G ~ Geometric(p) on {0,1,...}."""
    g = rng(seed).geometric(p, size=agents) - 1
    return np.minimum(g, cap).astype(np.int32)


def serve_batches(n_batches: int, seed: int, mean: int = 4096, lo: int = 64, hi: int = 65536) -> np.ndarray:
    """Batch sizes ceil(Exponential(mean)) clamped to [lo, hi]."""
    b = np.ceil(rng(seed).exponential(mean, size=n_batches)).astype(np.int64)
    return np.clip(b, lo, hi)


def serve_arrivals(n_batches: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Poisson arrival times (seconds from start) at ``rate_per_s`` batches/s."""
    gaps = rng(seed + 7).exponential(1.0 / rate_per_s, size=n_batches)
    return np.cumsum(gaps)


def op_script(n_ops: int, seed: int, lo: int = 1, hi: int = 8 * KiB, p_free: float = 0.4,
              p_invalid_size: float = 0.0) -> np.ndarray:
    """A mixed op list for single-thread replays: op >= 0 allocates op bytes;
    op < 0 frees the block allocated by op index (-op - 1).  Each live block
    is freed at most once."""
    g = rng(seed)
    ops = np.empty(n_ops, dtype=np.int64)
    live: list[int] = []
    for i in range(n_ops):
        if live and g.random() < p_free:
            j = live.pop(int(g.integers(len(live))))
            ops[i] = -j - 1
        else:
            if p_invalid_size and g.random() < p_invalid_size:
                ops[i] = 0 if g.random() < 0.5 else hi * 2
            else:
                ops[i] = int(math.floor(math.exp(g.uniform(math.log(lo), math.log(hi + 1)))))
                ops[i] = min(ops[i], hi)
            live.append(i)
    return ops


@dataclass
class ServePlan:
    """Batches of requests for the serving loop.  Requests are numbered in
    batch order; ops[i] >= 0 asks for that many bytes, ops[i] < 0 frees the
    block of request -ops[i]-1.  Batch b is requests [first[b], first[b+1])."""
    first: np.ndarray       # uint64, n_batches + 1
    ops: np.ndarray         # int64
    warm_batches: int       # leading batches that only allocate
    free_lag: int


def serve_plan(n_batches: int, seed: int, warm_requests: int, mean: int = 4096, lo: int = 64, hi: int = 65536,
               size_lo: int = 16, size_hi: int = 8 * KiB, p_free: float = 0.5, free_lag: int = 4) -> ServePlan:
    """Warm-up batches allocate until ``warm_requests`` allocations; after
    that each request is a free with probability ``p_free`` (while blocks are
    eligible), else an allocation.  A free picks uniformly among the live
    blocks allocated at least ``free_lag`` batches earlier; each block is
    freed at most once.  Batch sizes ceil(Exp(mean)) clamped to [lo, hi];
    allocation sizes log-uniform in [size_lo, size_hi]."""
    g = rng(seed + 11)
    bsz = serve_batches(n_batches, seed, mean, lo, hi)
    first = np.zeros(n_batches + 1, dtype=np.uint64)
    first[1:] = np.cumsum(bsz)
    total = int(first[-1])
    ops = np.empty(total, dtype=np.int64)
    pool = np.empty(total, dtype=np.int64)     # live ids eligible to be freed
    npool = 0
    allocs_of = []                               # alloc ids per batch
    n_alloc = 0
    warm = 0
    for b in range(n_batches):
        if b >= free_lag:
            add = allocs_of[b - free_lag]
            pool[npool:npool + len(add)] = add
            npool += len(add)
        f0, n = int(first[b]), int(bsz[b])
        warm_phase = n_alloc < warm_requests
        k = 0 if warm_phase else min(int(g.binomial(n, p_free)), npool)
        if warm_phase:
            warm += 1
        is_free = np.zeros(n, dtype=bool)
        if k:
            is_free[g.choice(n, k, replace=False)] = True
            pos = g.choice(npool, k, replace=False)
            targets = pool[pos].copy()
            # swap-remove the taken entries: holes outside the tail are
            # refilled with the tail entries that were not taken
            tail = npool - k
            in_tail = pos >= tail
            keep = np.ones(k, dtype=bool)
            keep[pos[in_tail] - tail] = False
            pool[pos[~in_tail]] = pool[tail:npool][keep]
            npool = tail
            ops[f0:f0 + n][is_free] = -targets - 1
        na = n - k
        ops[f0:f0 + n][~is_free] = sizes_log_uniform(na, size_lo, size_hi, seed + 100000 + b).astype(np.int64)
        ids = np.nonzero(~is_free)[0].astype(np.int64) + f0
        allocs_of.append(ids)
        n_alloc += na
    return ServePlan(first, ops, warm, free_lag)


def arrivals_ns(n_batches: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Poisson arrival times in nanoseconds from the start (first at 0)."""
    t = serve_arrivals(n_batches, rate_per_s, seed)
    t = t - t[0]
    return np.round(t * 1e9).astype(np.uint64)
