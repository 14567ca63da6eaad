"""CPU checks of bench.py's host logic: it refuses more than one GPU before
touching torch or the device, and it reports HBM traffic from the counter
record only while that record's source digest matches the kernel sources."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_digest_covers_each_kernel_source_in_order(bench):
    h = hashlib.sha256()
    for rel in bench.KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    assert bench.kernel_digest() == h.hexdigest()
    assert "paper_2504_18211_amd/csrc/hbheap.hip" in bench.KERNEL_SOURCES
    assert "include/hbheap_device.h" in bench.KERNEL_SOURCES


def _record(tmp_path, digest, traffic="123456"):
    p = tmp_path / "traffic.md"
    lines = ["# counters", "", "```"]
    if traffic is not None:
        lines.append(f"traffic_bytes_per_launch: {traffic}")
    lines += [f"kernel_source_sha256: {digest}", "```", ""]
    p.write_text("\n".join(lines))
    return str(p)


def test_traffic_reported_only_for_matching_digest(bench, tmp_path, monkeypatch):
    good = _record(tmp_path, bench.kernel_digest())
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", good)
    assert bench.recorded_traffic() == 123456.0

    stale = bench.kernel_digest()[:-1] + ("0" if bench.kernel_digest()[-1] != "0" else "1")
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, stale))
    assert bench.recorded_traffic() is None

    monkeypatch.setattr(bench, "TRAFFIC_RECORD", _record(tmp_path, bench.kernel_digest(), traffic=None))
    assert bench.recorded_traffic() is None

    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "missing.md"))
    assert bench.recorded_traffic() is None


def _synthetic_detail(bench):
    """A full-size record shaped like the bench's own (per-size, per-variant
    and per-load-point detail included), to size the summary line."""
    sizes = [16 << i for i in range(10)]
    per_size = {str(s): {"ok": 1 << 20, "alloc_us": 20.0, "free_us": 18.0, "first_alloc_us": 90.0,
                         "first_free_us": 30.0, "ops_per_s": 5.5e10,
                         "atomics_per_op_subsequent": {"alloc": {k: 0.1 for k in ("a", "b", "c", "d", "e")},
                                                       "free": {k: 0.1 for k in ("a", "b", "c", "d", "e")}}}
                for s in sizes}
    launches = [{"n": 1 << 20, "ok": 1 << 20, "t": 30e-6,
                 "atomics": {"state_ops": 32768, "headtail_ops": 16384, "pool_ops": 100, "spread_ops": 16384,
                             "slot_ops": 1 << 20}}] * 400
    ceil = {"same_address": 8e7, "lines_64": 2e9, "lines_1024": 8e9, "per_lane_random": 2.5e10,
            "xchg_contiguous": 2.3e11}
    rl = bench.alloc_roofline(launches, ceil, 12.0, 30421177.0)
    rl["kernel"] = "k_alloc_batch<false, 1u>"
    sweep = {"variant": "page", "shards": 64, "value": 3.8e10, "value_all_iterations": 2.6e10,
             "value_first_iteration": 9e9, "ms_per_step": 85.0, "wall_ops_per_s": 2.4e10,
             "batch_latency_us": {"alloc_p50": 21.0, "alloc_p99": 80.0, "free_p50": 17.0, "free_p99": 40.0},
             "per_size": per_size}
    head = dict(sweep, roofline=rl)
    serving = {"capacity_batches_per_s": 10000.0,
               "points": {p: {"served_ops_per_s": 4e7, "latency_us": {"p50": 200.0, "p99": 800.0},
                              "failed_requests": 0} for p in ("capacity", "load_0.25", "load_0.5", "load_0.9")}}
    growth = {"graph_ms": 0.28, "alloc_free_ops_per_s": 5e9,
              "autotune": {"best": {"chunk_bytes": 8192, "variant": "page", "width": 64, "eager_retirement": False},
                           "margin_vs_default": 1.0, "calibration_ms": {f"c{i}": 0.3 for i in range(84)}}}
    return {"metric": bench.METRIC, "value": 3.8e10, "unit": "ops/s", "n_gpus": 1, "steps": 3, "warmup": 1,
            "ms_per_step": 85.0, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic", "config": {"workload": "x" * 300, "variant": "page", "sizes": sizes},
            "headline": head, "other_variant": dict(sweep, variant="chunk"), "va_variant": dict(sweep, variant="va-page"),
            "va_chunk_variant": dict(sweep, variant="va-chunk"), "vl_variant": dict(sweep, variant="vl-page"),
            "vl_chunk_variant": dict(sweep, variant="vl-chunk"), "eager_chunk_variant": dict(sweep, variant="chunk-eager"),
            "ablation_width1": {"value": 1.8e9}, "vs_plain": 1000.0,
            "plain": {"value": 3e7, "ours_same_sizes": 3.8e10, "iterations": 10, "threads": 1 << 20,
                      "null_requests": 0, "mismatches": 0, "sizes": {str(s): {"alloc_us": [1.0] * 10} for s in sizes}},
            "cpu_baseline": {"value": 1e8, "unit": "ops/s", "cores": 1, "kind": "oracle", "sample": "y" * 150,
                             "cpu_model": "z"},
            "paper_sweeps": {"size_sweep_1024_allocs": {v: per_size for v in "abcdef"}},
            "growth": growth, "serving": serving, "detail_path": "gpurun_out/bench_detail.json"}


def test_summary_line_is_compact_and_carries_the_contract_fields(bench):
    import json
    d = _synthetic_detail(bench)
    line = json.dumps(bench.compact(d))
    assert len(json.dumps(d)) > 20000          # the detail alone would not fit the driver's tail
    assert len(line) < 4096
    s = json.loads(line)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "vs_plain",
              "value_all_iterations", "serving"):
        assert k in s, k
    rl = s["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in rl, k
    assert rl["bound"] == "hbm" and rl["unit"] == "GB/s" and rl["peak"] == 8000.0
    assert s["cpu_baseline"]["kind"] == "oracle" and s["cpu_baseline"]["cores"] == 1
    assert s["serving"]["load_0.9"]["p99_us"] == 800.0
    assert set(s["variants_ops_per_s"]) == {"chunk", "va-page", "va-chunk", "vl-page", "vl-chunk", "chunk-eager",
                                            "width1"}


def test_roofline_fractions(bench):
    # one launch of 2^20 requests, all served, in 30 us: 24 B per request
    n = 1 << 20
    ceil = {"lines_64": 2e9, "per_lane_random": 2.5e10, "xchg_contiguous": 2e11}
    at = {"state_ops": 2000, "headtail_ops": 1000, "pool_ops": 0, "spread_ops": 25000, "slot_ops": n}
    rl = bench.alloc_roofline([{"n": n, "ok": n, "t": 30e-6, "atomics": at}], ceil, 12.0, None)
    assert rl["algorithmic_bytes_per_launch"] == 24 * n
    assert abs(rl["achieved"] - 24 * n / 30e-6 / 1e9) < 1e-6
    assert abs(rl["frac"] - rl["achieved"] / 8000.0) < 1e-12
    t_at = 3000 / 2e9 + 25000 / 2.5e10 + n / 2e11
    assert abs(rl["atomic"]["frac"] - t_at / 30e-6) < 1e-9
    assert abs(rl["latency"]["frac"] - 12.0 / 30.0) < 1e-12
    assert rl["binding"] == "latency"
    # half the requests fail: 16 B each, no slot traffic
    rl = bench.alloc_roofline([{"n": n, "ok": n // 2, "t": 30e-6, "atomics": at}], ceil, 1.0, None)
    assert rl["algorithmic_bytes_per_launch"] == 16 * n + 8 * (n // 2)
