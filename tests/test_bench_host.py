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
