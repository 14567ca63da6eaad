"""CPU checks of the seeded workload generators: each draws what its recipe
states (ranges, proportions, closed-form means), and the serving plans are
valid request lists (every free names an earlier allocation at least
`free_lag` batches back, each block is freed at most once)."""
import math

import numpy as np

from paper_2504_18211_amd import inputs


def test_log_uniform_range_and_median():
    s = inputs.sizes_log_uniform(200000, 4, 8192, 1)
    assert s.min() >= 4 and s.max() <= 8192
    # median of exp(U[ln 4, ln 8193)) is sqrt(4 * 8193); floor shifts it down by < 1
    med = float(np.median(s))
    assert abs(med - math.sqrt(4 * 8193)) < 0.03 * math.sqrt(4 * 8193)


def test_growth_doublings_distribution():
    d = inputs.growth_doublings(1 << 18, inputs.SEED_GROWTH)
    assert d.min() >= 0 and d.max() <= 8
    # min(8, G), G ~ Geometric(0.3) on {0, 1, ...}: P(T >= s) = 0.7^s for s <= 8
    for s in range(1, 9):
        assert abs((d >= s).mean() - 0.7 ** s) < 0.01
    assert abs(d.mean() - sum(0.7 ** s for s in range(1, 9))) < 0.02


def test_churn_round_frees_half_without_repeats():
    idx, sizes = inputs.churn_round(1 << 16, 3, inputs.SEED_CHURN)
    assert len(idx) == 1 << 15 and len(np.unique(idx)) == len(idx)
    assert (np.diff(idx) > 0).all() and sizes.min() >= 4 and sizes.max() <= 8192


def test_serve_batches_clamped_exponential():
    b = inputs.serve_batches(100000, inputs.SEED_SERVE)
    assert b.min() >= 64 and b.max() <= 65536
    # clamping at 64 raises the mean of Exp(4096) by 64 * P(X < 64) - E[X; X < 64] (small)
    assert abs(b.mean() - 4096) < 0.03 * 4096


def test_serve_plan_is_a_valid_request_list():
    plan = inputs.serve_plan(400, 7, warm_requests=200000, mean=1024, lo=64, hi=8192, free_lag=3)
    first, ops = plan.first, plan.ops
    assert first[0] == 0 and first[-1] == len(ops) and (np.diff(first.astype(np.int64)) >= 64).all()
    batch_of = np.searchsorted(first, np.arange(len(ops)), side="right") - 1
    fr = np.nonzero(ops < 0)[0]
    tg = -ops[fr] - 1
    assert (ops[tg] >= 0).all(), "a free names a free"
    assert len(np.unique(tg)) == len(tg), "a block freed twice"
    assert (batch_of[tg] + plan.free_lag <= batch_of[fr]).all(), "a free too close to its allocation"
    # warm-up batches only allocate, until the requested count
    wb = plan.warm_batches
    assert (ops[: first[wb]] >= 0).all() and first[wb - 1] < 200000 <= first[wb]
    # after the warm-up about half of the requests are frees
    mixed = ops[first[wb]:]
    assert abs((mixed < 0).mean() - 0.5) < 0.02
    sizes = ops[ops >= 0]
    assert sizes.min() >= 16 and sizes.max() <= 8192


def test_arrivals_poisson_rate():
    a = inputs.arrivals_ns(20001, 5000.0, 3)
    assert a[0] == 0 and (np.diff(a.astype(np.int64)) >= 0).all()
    # 20000 gaps of mean 1/5000 s
    assert abs(float(a[-1]) * 1e-9 - 4.0) < 0.1
