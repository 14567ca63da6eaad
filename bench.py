#!/usr/bin/env python3
"""Benchmark of the device heap allocator on one MI355X.

Workload (the headline): a 4 GiB heap of 8 KiB chunks; 2^20 threads, one
fixed request size per launch, swept over powers of two 16 B .. 8 KiB.  One
step = for every size: ten iterations of an allocation launch, a payload
write, a read-back check and a free launch (the paper's driver loop,
Methods), then a quiescent trim before the next size.  As in the paper, the
allocator's figure is the time of the allocations and frees averaged over
the iterations after the first ("subsequent iterations", Methods): value =
successful (alloc + free) ops / alloc+free launch time over iterations
2..10 (HIP events on the launch stream); iterations 1..10 are reported too,
and the first iteration of each size (served by refills of a freshly
trimmed heap) on its own.  Each size's ten iterations are queued behind a
short device-side wait, so every event pair times its launch on the
device's timeline rather than the host's submission latency.  The whole
step's wall time (payload write/check, those waits and trims included) is
ms_per_step, and all ops over it is wall_ops_per_s.

The headline runs the page-queue variant (the faster one on this workload);
the other queue variants run the same sweep for one step beside it.

Also measured in the same process:
  * device ceilings: atomics on one address, on 64 and 1024 lines, on
    per-lane random words, lane-contiguous exchanges, a chain of dependent
    round trips, and an HBM copy;
  * a counting pass with the heap's statistics flag, giving the exact
    atomics issued per launch by target;
  * the roofline of the allocation kernel: HBM bytes (algorithmic, per
    launch) against 8 TB/s, its atomics priced at the ceiling whose address
    pattern matches each kind, and the latency floor of its chain of
    dependent round trips; which of the three binds;
  * the plain baseline: the runtime's own per-thread device malloc/free in
    the same driver loop;
  * the CPU baseline: the sequential oracle on a bounded sample, one core.

roofline.traffic is the HBM bytes per allocation launch (FETCH_SIZE and
WRITE_SIZE counters, scaled by the same counters' reading for a copy of known
size) recorded in the counter summary under profiles/; it is null once the
kernel sources differ from the digest stored there.

Output: the last stdout line is one compact JSON object (a few KB) with the
headline and a summary of every other line; the full record (per size, per
variant, per load point) goes to --detail PATH, or to stderr as one line
starting with "detail " when no path is given.  Only --gpus 1 is supported.
`--copy-probe BYTES` only runs the HBM copy kernel (to calibrate traffic
counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "device malloc+free ops/sec (2^20 threads, 16B-8KiB) vs plain; p99 batch latency"
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published
# Algorithmic HBM bytes of one allocation launch of the batch interface: per
# request the 8 B size read and the 8 B pointer write; per page served from
# a queue, its 4 B slot read and then reset to the empty mark.
ALG_IO_BYTES = 16
ALG_SERVED_BYTES = 8
# Dependent device round trips per wave on the page variant's fast path
# (queues already stocked): the request size (with the pool hint beside it),
# the class state word, the head word, the slot.
FAST_PATH_ROUND_TRIPS = 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=10, help="alloc-write-check-free iterations per size")
    ap.add_argument("--variant", choices=["chunk", "page", "va-page", "va-chunk", "vl-page", "vl-chunk"],
                    default="page")
    ap.add_argument("--width", type=int, default=64)
    ap.add_argument("--rows", type=int, default=0, help="requests per lane of the batch kernels (0: the library's 4)")
    ap.add_argument("--shards", type=int, default=0, help="queue shards (0: one per 256 chunks, up to 64)")
    ap.add_argument("--detail", type=str, default="", help="write the full JSON record here (else to stderr)")
    ap.add_argument("--no-other", action="store_true", help="skip the other queue variant")
    ap.add_argument("--no-va", action="store_true", help="skip the virtualised-array and -list variant lines")
    ap.add_argument("--no-eager", action="store_true", help="skip the eager chunk retirement line")
    ap.add_argument("--no-ablation", action="store_true", help="skip the width-1 (no aggregation) ablation")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain device-malloc baseline")
    ap.add_argument("--plain-iters", type=int, default=10, help="driver-loop iterations of the plain baseline")
    ap.add_argument("--plain-sizes", type=str, default="16,32,64,128,256,512,1024,2048",
                    help="sizes of the plain baseline (at 2^20 threads one iteration takes 44 s at 4 KiB, so the "
                         "default run stops at 2 KiB)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-host-malloc", action="store_true",
                    help="skip the host C library malloc/free context figure")
    ap.add_argument("--host-malloc-iters", type=int, default=3,
                    help="rounds per size of the host malloc/free context figure (the first is not counted)")
    ap.add_argument("--sizes", type=str, default="", help="comma list overriding the 16..8192 sweep")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run an HBM copy of this many bytes")
    ap.add_argument("--no-growth", action="store_true", help="skip the growth line (graph replay, autotuner)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving line")
    ap.add_argument("--no-paper-sweeps", action="store_true", help="skip the paper's size and thread sweeps")
    ap.add_argument("--growth-reps", type=int, default=20)
    ap.add_argument("--serve-batches", type=int, default=10000, help="mixed batches per load point")
    ap.add_argument("--serve-slots", type=int, default=4)
    return ap.parse_args(argv)


# sources that make up the allocation kernel; the traffic recorded with the
# hardware counters is only reported while their digest is unchanged
KERNEL_SOURCES = ("paper_2504_18211_amd/csrc/hbheap.hip", "include/hbheap_device.h", "include/hbheap_types.h")
TRAFFIC_RECORD = "profiles/k_alloc_batch_sweep_4GiB_page_traffic.md"


def kernel_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per allocation launch from the counter summary, or None when
    there is none or the kernel sources changed since it was taken."""
    try:
        text = open(os.path.join(ROOT, TRAFFIC_RECORD)).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith(("traffic_bytes_per_launch", "kernel_source_sha256")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_digest() or "traffic_bytes_per_launch" not in kv:
        return None
    return float(kv["traffic_bytes_per_launch"])


def head_rows_of(args, variant: int, width: int | None = None) -> int:
    """Requests per lane of the allocation kernel the library launches for
    this heap: its rows (4 by default) for every variant but the
    virtualised-list page variant, at width 16 or more, else one."""
    width = args.width if width is None else width
    return (args.rows or 4) if variant != 4 and width >= 16 else 1


def alloc_roofline(launches, ceilings, chain_us, traffic):
    """Roofline of the allocation kernel from its launches (per launch: the
    requests n, the successful ones ok, the event-timed seconds t, the
    counting pass's atomics by target for that launch's iteration kind).

    Three bounds, each as the fraction of the launch time it would need:
      * HBM: algorithmic bytes per launch (16 B per request, plus 8 B per
        served page) against 8 TB/s;
      * atomics: every atomic priced at the measured ceiling whose address
        pattern matches it -- state, head/tail and pool words (one line per
        shard and class) at the 64-line rate, ring slots (a wave on
        consecutive words) at the lane-contiguous exchange rate, bitmask
        and count words at the per-lane random rate;
      * latency: the measured time of a kernel of the same number of waves
        that runs the fast path's dependent round trips and nothing else.
    The contract fields (bound/achieved/peak/unit/frac) report HBM; which of
    the three is nearest its ceiling is `binding`."""
    t_sum = sum(x["t"] for x in launches)
    nl = len(launches)
    alg_bytes = sum(ALG_IO_BYTES * x["n"] + ALG_SERVED_BYTES * x["ok"] for x in launches)
    achieved = alg_bytes / t_sum / 1e9
    price = {"state_ops": ceilings["lines_64"], "headtail_ops": ceilings["lines_64"],
             "pool_ops": ceilings["lines_64"], "slot_ops": ceilings["xchg_contiguous"],
             "spread_ops": ceilings["per_lane_random"]}
    t_atomic = 0.0
    per_kind = {k: 0 for k in price}
    for x in launches:
        for k, r in price.items():
            c = x["atomics"].get(k, 0)
            per_kind[k] += c
            t_atomic += c / r
    avg = t_sum / nl
    frac_hbm = achieved / HBM_PEAK_GBPS
    frac_atomic = t_atomic / t_sum
    frac_latency = chain_us * 1e-6 / avg
    binding = max((("hbm", frac_hbm), ("atomic", frac_atomic), ("latency", frac_latency)), key=lambda kv: kv[1])[0]
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": frac_hbm,
        "traffic": traffic,
        "binding": binding,
        "algorithmic_bytes_per_launch": alg_bytes / nl,
        "avg_launch_us": avg * 1e6,
        "launches": nl,
        "atomic": {"frac": frac_atomic,
                   "per_launch": {k: v / nl for k, v in per_kind.items()},
                   "ceilings_g_per_s": {k: r / 1e9 for k, r in price.items()}},
        "latency": {"frac": frac_latency, "floor_us": chain_us, "round_trips": FAST_PATH_ROUND_TRIPS},
    }


def compact(d: dict) -> dict:
    """The one-line summary printed last on stdout (the driver keeps only the
    tail of the output): the headline, its roofline and baselines, and one
    figure per other line.  The full record is d itself."""
    def r(x, nd=4):
        if x is None:
            return None
        return float(f"{x:.{nd}g}")

    head = d["headline"]
    rl = head.get("roofline") or {}
    out = {k: d[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                             "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config")}
    out["value_all_iterations"] = head["value_all_iterations"]
    out["first_iteration_ops_per_s"] = head.get("value_first_iteration")
    out["alloc_us_by_size"] = {s: {"first": v["first_alloc_us"], "later": v["alloc_us"]}
                               for s, v in head["per_size"].items()}
    out["free_us_by_size"] = {s: v["free_us"] for s, v in head["per_size"].items()}
    out["wall_ops_per_s"] = head["wall_ops_per_s"]
    out["batch_latency_us"] = {k: r(v) for k, v in head["batch_latency_us"].items()}
    if rl:
        out["roofline"] = {
            "bound": rl["bound"], "achieved": r(rl["achieved"]), "peak": rl["peak"], "unit": rl["unit"],
            "frac": r(rl["frac"]), "traffic": rl["traffic"], "kernel": rl.get("kernel"),
            "binding": rl["binding"], "avg_launch_us": r(rl["avg_launch_us"]),
            "algorithmic_bytes_per_launch": r(rl["algorithmic_bytes_per_launch"]),
            "atomic_frac": r(rl["atomic"]["frac"]), "latency_frac": r(rl["latency"]["frac"]),
            "latency_floor_us": r(rl["latency"]["floor_us"]),
        }
    cpu = d.get("cpu_baseline")
    out["cpu_baseline"] = ({k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")} if cpu else None)
    hm = d.get("host_malloc_context")
    if hm:
        out["host_malloc_context"] = {"value": r(hm["value"]), "threads": hm["threads"], "failed": hm["failed"],
                                      "cpu_model": hm["cpu_model"]}
    plain = d.get("plain")
    out["vs_plain"] = r(d.get("vs_plain"))
    if plain:
        out["plain"] = {"value": r(plain.get("value")), "ours_same_sizes": r(plain.get("ours_same_sizes")),
                        "iterations": plain.get("iterations"), "threads": plain.get("threads"),
                        "sizes": [int(x) for x in plain.get("sizes", {})], "not_run": plain.get("not_run"),
                        "null_requests": plain.get("null_requests"), "mismatches": plain.get("mismatches")}
    variants = {}
    for name, key in (("chunk", "other_variant"), ("va-page", "va_variant"), ("va-chunk", "va_chunk_variant"),
                      ("vl-page", "vl_variant"), ("vl-chunk", "vl_chunk_variant"),
                      ("chunk-eager", "eager_chunk_variant")):
        v = d.get(key)
        if v:
            variants[v.get("variant", name) if key != "eager_chunk_variant" else name] = r(v["value"])
    ab = d.get("ablation_width1")
    if ab:
        variants["width1"] = r(ab["value"])
    out["variants_ops_per_s"] = variants
    sv = d.get("serving")
    if sv and "points" in sv:
        out["serving"] = {"capacity_batches_per_s": r(sv["capacity_batches_per_s"]),
                          "capacity_ops_per_s": r(sv["points"]["capacity"]["served_ops_per_s"])}
        for f in ("0.25", "0.5", "0.9"):
            p = sv["points"].get(f"load_{f}")
            if p:
                out["serving"][f"load_{f}"] = {"p50_us": r(p["latency_us"]["p50"]), "p99_us": r(p["latency_us"]["p99"]),
                                               "failed": p["failed_requests"]}
    g = d.get("growth")
    if g and "graph_ms" in g:
        out["growth"] = {"graph_ms": r(g["graph_ms"]), "alloc_free_ops_per_s": r(g["alloc_free_ops_per_s"]),
                         "pick": g["autotune"]["best"], "margin_vs_default": r(g["autotune"]["margin_vs_default"])}
    out["detail"] = d.get("detail_path")
    return out


_SLEEP_CYCLES_PER_US = None


def hold_stream(torch, us: float = 1000.0):
    """Queue a device-side wait of about `us` microseconds on the current
    stream, so that the host enqueues the launches that follow before the
    device reaches them.  Each launch is then timed by its own event pair on
    the device's timeline without the host's submission latency (the device
    would otherwise sit idle between an event and the launch it brackets,
    whenever Python submits more slowly than the kernels run)."""
    global _SLEEP_CYCLES_PER_US
    if _SLEEP_CYCLES_PER_US is None:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda._sleep(1000)
        e0.record()
        torch.cuda._sleep(1_000_000)
        e1.record()
        torch.cuda.synchronize()
        _SLEEP_CYCLES_PER_US = 1_000_000 / max(1.0, e0.elapsed_time(e1) * 1e3)
    torch.cuda._sleep(int(us * _SLEEP_CYCLES_PER_US))


VNAMES = ("chunk", "page", "va-page", "va-chunk", "vl-page", "vl-chunk")


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a, dtype=float), q)) if len(a) else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the heap lives in one GPU's HBM and "
              "every allocation is served on that GPU; there is no multi-GPU path to measure.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2504_18211_amd import hbheap as hb
    from paper_2504_18211_amd import inputs

    hb.lib()  # fails loudly without the built library
    VARIANTS = {"chunk": hb.VARIANT_CHUNK, "page": hb.VARIANT_PAGE, "va-page": hb.VARIANT_VA_PAGE,
                "va-chunk": hb.VARIANT_VA_CHUNK, "vl-page": hb.VARIANT_VL_PAGE, "vl-chunk": hb.VARIANT_VL_CHUNK,
                "chunk-eager": hb.VARIANT_CHUNK}
    # creation flags per line: eager chunk retirement is fixed at creation
    CREATE_FLAGS = {"chunk-eager": hb.FLAG_EAGER}
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(3)
    dev = torch.device("cuda:0")

    def ev():
        return torch.cuda.Event(enable_timing=True)

    if args.copy_probe:
        nbytes = args.copy_probe // 16 * 16
        a = torch.ones(nbytes, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        ts = []
        for _ in range(2):
            e0, e1 = ev(), ev()
            e0.record()
            hb.hb_stream_copy(b, a, nbytes)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 2,
                          "gb_per_s": 2 * nbytes / min(ts) / 1e9}), flush=True)
        return

    w = inputs.SWEEP
    n = w.threads
    sizes_list = [int(x) for x in args.sizes.split(",")] if args.sizes else list(inputs.SWEEP_SIZES)

    # ---------------- device ceilings ----------------
    probe_buf = torch.zeros(64 << 20, dtype=torch.uint8, device=dev)

    def probe_time(pattern, lines, threads, iters, reps=3):
        best = None
        for _ in range(reps):
            e0, e1 = ev(), ev()
            hold_stream(torch, 200.0)
            e0.record()
            hb.hb_atomic_probe(pattern, probe_buf, probe_buf.numel(), threads, lines, iters)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3
            best = t if best is None else min(best, t)
        return best

    def probe(pattern, lines, threads, iters):
        n_at = threads * iters if pattern in (2, 4, 5, 6, 7, 8) else threads // 64 * iters
        return n_at / probe_time(pattern, lines, threads, iters)

    # what an event pair adds around a launch: median over a one-wave kernel
    # doing a single atomic
    def event_overhead_us():
        """An event pair around a minimal launch, queued behind a device wait
        as the timed launches are: dispatch plus event packets."""
        buf = torch.zeros(1 << 16, dtype=torch.uint8, device=dev)
        hold_stream(torch)
        es = []
        for _ in range(50):
            e0, e1 = ev(), ev()
            e0.record()
            hb.hb_atomic_probe(1, buf, buf.numel(), 64, 1, 1)
            e1.record()
            es.append((e0, e1))
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) * 1e3 for e0, e1 in es]))

    ev_overhead = event_overhead_us()
    ceilings = {
        "same_address": probe(0, 1, 1 << 20, 4),
        "lines_64": probe(1, 64, 1 << 20, 4),
        "lines_1024": probe(1, 1024, 1 << 20, 4),
        "per_lane_random": probe(2, 1, 1 << 20, 4),
        "xchg_contiguous": probe(5, 1, 1 << 20, 4),
    }
    # latency floor: the allocation kernel's launch shape (one lane per
    # `rows` requests, 256-lane blocks), each lane running the fast path's
    # dependent round trips (a lane's rows share every round trip)
    head_rows = head_rows_of(args, VARIANTS[args.variant])
    chain_us = probe_time(8, 1, n // head_rows, FAST_PATH_ROUND_TRIPS, reps=5) * 1e6
    chain1_us = probe_time(8, 1, n // head_rows, 1, reps=5) * 1e6
    a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    tc = []
    for _ in range(3):
        e0, e1 = ev(), ev()
        e0.record()
        hb.hb_stream_copy(b, a, a.numel())
        e1.record()
        torch.cuda.synchronize()
        tc.append(e0.elapsed_time(e1) / 1e3)
    copy_gbps = 2 * a.numel() / min(tc) / 1e9
    del a, b
    log("ceilings: " + ", ".join(f"{k} {v/1e9:.2f} G/s" for k, v in ceilings.items()) +
        f"; chain of {FAST_PATH_ROUND_TRIPS} round trips {chain_us:.1f} us (1: {chain1_us:.1f} us); "
        f"copy {copy_gbps:.0f} GB/s")

    size_dev = {s: torch.from_numpy(inputs.sizes_fixed(n, s).view(np.int64)).to(dev) for s in sizes_list}
    ptrs = torch.zeros(n, dtype=torch.int64, device=dev)
    mism = torch.zeros(1, dtype=torch.int64, device=dev)
    keys = ("state_ops", "headtail_ops", "pool_ops", "spread_ops", "slot_ops")

    def run_sweep(variant_name: str, steps: int, warmup: int, count: bool, width: int | None = None) -> dict:
        variant = VARIANTS[variant_name]
        heap = hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant, width=args.width if width is None else width,
                       shards=args.shards, flags=CREATE_FLAGS.get(variant_name, 0), rows=args.rows)
        shards = int(heap.info.n_shards)

        def one_size(s, rec):
            sd = size_dev[s]
            hold_stream(torch)
            for it in range(args.iters):
                e = [ev() for _ in range(4)]
                e[0].record()
                heap.alloc(sd, ptrs)
                e[1].record()
                hb.heap_pattern_write(heap.h, ptrs, sd, w.seed)
                hb.heap_pattern_check(heap.h, ptrs, sd, w.seed, mism)
                ok = (ptrs != 0).sum()
                e[2].record()
                heap.free(ptrs)
                e[3].record()
                rec.append((s, it, e, ok))
            heap.trim()

        def run_step(rec):
            for s in sizes_list:
                one_size(s, rec)

        # counting pass: exact atomics per launch by target, for the first
        # iteration after a trim and for a subsequent one
        counts = {}
        if count:
            heap.set_flags(hb.FLAG_STATS)
            for s in sizes_list:
                sd = size_dev[s]
                counts[s] = {}
                for phase in ("first", "subsequent"):
                    before = heap.stats()
                    heap.alloc(sd, ptrs)
                    torch.cuda.synchronize()
                    mid = heap.stats()
                    heap.free(ptrs)
                    torch.cuda.synchronize()
                    after = heap.stats()
                    counts[s][phase] = {"alloc": {k: mid[k] - before[k] for k in keys},
                                        "free": {k: after[k] - mid[k] for k in keys}}
                heap.trim()
            heap.set_flags(0)
            assert heap.error() == 0, "heap error during counting pass"

        warm = []
        for _ in range(warmup):
            run_step(warm)
        torch.cuda.synchronize()
        recs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            run_step(recs)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0

        if int(mism.item()) != 0:
            log(f"PAYLOAD MISMATCHES: {int(mism.item())}")
            sys.exit(4)
        err = heap.error()
        heap.close()
        if err:
            log(f"HEAP ERROR WORD {err:#x}")
            sys.exit(5)

        per_size = {s: {"alloc_us": [], "free_us": [], "first_alloc_us": [], "first_free_us": [], "ok": 0}
                    for s in sizes_list}
        sub_ops = sub_t = all_ops = all_t = first_ops = first_t = 0.0
        t_alloc_sub, t_free_sub = [], []
        for s, it, e, ok in recs:
            ta = e[0].elapsed_time(e[1]) / 1e3
            tf = e[2].elapsed_time(e[3]) / 1e3
            okv = int(ok.item())
            all_ops += 2 * okv
            all_t += ta + tf
            if it > 0:
                sub_ops += 2 * okv
                sub_t += ta + tf
                t_alloc_sub.append(ta)
                t_free_sub.append(tf)
                per_size[s]["alloc_us"].append(ta * 1e6)
                per_size[s]["free_us"].append(tf * 1e6)
            else:
                first_ops += 2 * okv
                first_t += ta + tf
                per_size[s]["first_alloc_us"].append(ta * 1e6)
                per_size[s]["first_free_us"].append(tf * 1e6)
            per_size[s]["ok"] = okv
        out = {
            "variant": variant_name,
            "shards": shards,
            "value": sub_ops / sub_t,
            "value_all_iterations": all_ops / all_t,
            "value_first_iteration": first_ops / first_t if first_t else None,
            "ms_per_step": wall / steps * 1e3,
            "wall_ops_per_s": all_ops / wall,
            "batch_latency_us": {
                "alloc_p50": pct(t_alloc_sub, 50) * 1e6, "alloc_p99": pct(t_alloc_sub, 99) * 1e6,
                "free_p50": pct(t_free_sub, 50) * 1e6, "free_p99": pct(t_free_sub, 99) * 1e6,
            },
            "per_size": {
                str(s): {
                    "ok": v["ok"],
                    "alloc_us": round(float(np.mean(v["alloc_us"])), 1),
                    "free_us": round(float(np.mean(v["free_us"])), 1),
                    "first_alloc_us": round(float(np.mean(v["first_alloc_us"])), 1),
                    "first_free_us": round(float(np.mean(v["first_free_us"])), 1),
                    "ops_per_s": round(2 * v["ok"] / ((np.mean(v["alloc_us"]) + np.mean(v["free_us"])) * 1e-6), 0),
                }
                for s, v in per_size.items()
            },
        }
        if count:
            for s in sizes_list:
                out["per_size"][str(s)]["atomics_per_op_subsequent"] = {
                    ph: {k: round(c / max(1, per_size[s]["ok"]), 4) for k, c in counts[s]["subsequent"][ph].items()}
                    for ph in ("alloc", "free")}
            # roofline of the dominant kernel, k_alloc_batch, over every
            # non-counting allocation launch of this sweep (warmup + timed:
            # the population a kernel trace averages over)
            launches = []
            for s, it, e, ok in warm + recs:
                launches.append({"n": n, "ok": int(ok.item()), "t": e[0].elapsed_time(e[1]) / 1e3,
                                 "atomics": counts[s]["first" if it == 0 else "subsequent"]["alloc"]})
            rl = alloc_roofline(launches, ceilings, chain_us, recorded_traffic())
            # the library's kernel instance: the variant's, or 6 for the chunk
            # variant with eager retirement
            inst = 6 if CREATE_FLAGS.get(variant_name, 0) & hb.FLAG_EAGER else variant
            rl["kernel"] = f"k_alloc_batch<false, {inst}u, {head_rows_of(args, variant, width)}u>"
            rl["event_overhead_us"] = ev_overhead
            state_atomics = sum(x["atomics"]["state_ops"] for x in launches)
            t_sum = sum(x["t"] for x in launches)
            busiest = state_atomics / shards / t_sum
            rl["busiest_word"] = {"achieved_g_per_s": busiest / 1e9, "peak_g_per_s": ceilings["same_address"] / 1e9,
                                  "frac": busiest / ceilings["same_address"], "shards": shards}
            rl["alloc_share_of_alloc_free_time"] = sum(t_alloc_sub) / (sum(t_alloc_sub) + sum(t_free_sub))
            out["roofline"] = rl
        return out

    head = run_sweep(args.variant, args.steps, args.warmup, count=True)
    log(f"{args.variant}: {head['value']/1e9:.2f} G ops/s (iterations 2..10), first iterations "
        f"{(head['value_first_iteration'] or 0)/1e9:.2f} G ops/s; roofline: HBM frac {head['roofline']['frac']:.3f}, "
        f"atomic frac {head['roofline']['atomic']['frac']:.3f}, latency frac {head['roofline']['latency']['frac']:.3f} "
        f"(binding: {head['roofline']['binding']})")

    other = None
    if not args.no_other:
        other_name = "chunk" if args.variant != "chunk" else "page"
        other = run_sweep(other_name, 1, 1, count=False)
        log(f"{other_name}: {other['value']/1e9:.2f} G ops/s (iterations 2..10)")
    # the page variant with its queues in virtualised arrays (one slot budget
    # per shard, shared by the classes in segments), one step
    # the paper's virtualised variants: queues in segments drawn from a
    # per-shard store, found through a directory (va) or a linked list (vl);
    # one step each
    virt = {}
    if not args.no_va:
        for name in ("va-page", "va-chunk", "vl-page", "vl-chunk"):
            if name == args.variant:
                continue
            virt[name] = run_sweep(name, 1, 1, count=False)
            log(f"{name}: {virt[name]['value']/1e9:.2f} G ops/s (iterations 2..10)")
    va, va_chunk = virt.get("va-page"), virt.get("va-chunk")

    # eager chunk retirement (chunk variant: a chunk whose pages are all free
    # returns to its shard's pool at once): the same sweep, one step -- every
    # free launch retires the chunks it empties and the next allocation
    # takes them back from the pool rings; then a change of class with no
    # trim, lazy against eager
    eager = None
    if not args.no_eager:
        eager = run_sweep("chunk-eager", 1, 1, count=True)
        # its own roofline (atomics counted in its counting pass); the
        # recorded HBM traffic belongs to the headline's page instance
        eager["roofline"]["traffic"] = None
        log(f"chunk-eager: {eager['value']/1e9:.2f} G ops/s (iterations 2..10), roofline: HBM frac "
            f"{eager['roofline']['frac']:.3f}, atomic frac {eager['roofline']['atomic']['frac']:.3f}, latency frac "
            f"{eager['roofline']['latency']['frac']:.3f}")
        eager["class_change"] = {}
        for name, fl in (("lazy", 0), ("eager", hb.FLAG_EAGER)):
            heap = hb.Heap(w.heap_bytes, w.chunk_bytes, variant=hb.VARIANT_CHUNK, shards=args.shards, flags=fl)
            rec = {}
            for phase, s in (("fill_4KiB", 4096), ("refill_16B", 16)):
                hold_stream(torch)
                e = [ev() for _ in range(4)]
                e[0].record()
                heap.alloc(size_dev[s], ptrs)
                e[1].record()
                ok = int((ptrs != 0).sum().item())
                e[2].record()
                heap.free(ptrs)
                e[3].record()
                torch.cuda.synchronize()
                rec[phase] = {"ok": ok, "alloc_us": e[0].elapsed_time(e[1]) * 1e3,
                              "free_us": e[2].elapsed_time(e[3]) * 1e3}
            err = heap.error()
            heap.close()
            if err:
                log(f"HEAP ERROR WORD {err:#x}")
                sys.exit(5)
            eager["class_change"][name] = rec
            log(f"class change {name}: 4 KiB ok {rec['fill_4KiB']['ok']}, then 16 B ok {rec['refill_16B']['ok']} "
                f"(no trim)")
        # fragmentation under a shifting mix: the churn heap (8 GiB, 2^21
        # blocks, log-uniform 4 B .. 8 KiB); each round frees a random half
        # and reallocates it with sizes alternating between small (4 .. 256 B)
        # and large (1 .. 8 KiB); chunks in use after each round (exact: the
        # pools' counters at quiescence), lazy against eager
        wc = inputs.CHURN
        nc = wc.threads
        eager["shifting_churn"] = {"workload": f"{wc.heap_bytes >> 30} GiB heap, {nc} blocks, rounds of half freed "
                                               "and reallocated, sizes alternating 4..256 B / 1..8 KiB",
                                   "n_chunks": wc.heap_bytes // wc.chunk_bytes}
        for name, fl in (("lazy", 0), ("eager", hb.FLAG_EAGER)):
            heap = hb.Heap(wc.heap_bytes, wc.chunk_bytes, variant=hb.VARIANT_CHUNK, shards=args.shards, flags=fl)
            szh = inputs.sizes_log_uniform(nc, 4, 8 * 1024, wc.seed)
            sz = torch.from_numpy(szh.view(np.int64)).to(dev)
            pp = torch.zeros(nc, dtype=torch.int64, device=dev)
            heap.alloc(sz, pp)
            gen = torch.Generator(device=dev)
            gen.manual_seed(wc.seed)
            traj, nulls, live = [], [], []
            for r in range(10):
                idx = torch.randperm(nc, device=dev, generator=gen)[: nc // 2]
                heap.free(pp[idx].contiguous())
                lo, hi = (4, 256) if r % 2 == 0 else (1024, 8 * 1024)
                nsz = torch.from_numpy(inputs.sizes_log_uniform(nc // 2, lo, hi, wc.seed + 1 + r).view(np.int64)).to(dev)
                sz[idx] = nsz
                npp = torch.zeros(nc // 2, dtype=torch.int64, device=dev)
                heap.alloc(nsz, npp)
                pp[idx] = npp
                ok = pp != 0
                cls_bytes = torch.clamp(sz, min=16)
                cls_bytes = torch.pow(2, torch.ceil(torch.log2(cls_bytes.double()))).long()
                live.append(int((cls_bytes * ok).sum().item()))
                nulls.append(int((npp == 0).sum().item()))
                traj.append(hb.heap_chunks_in_use(heap.h))
            err = heap.error()
            heap.close()
            if err:
                log(f"HEAP ERROR WORD {err:#x}")
                sys.exit(5)
            eager["shifting_churn"][name] = {"chunks_in_use": traj, "failed_requests": nulls, "live_page_bytes": live}
            log(f"shifting churn {name}: chunks in use {traj[-1]} of {wc.heap_bytes // wc.chunk_bytes}, "
                f"failed requests {sum(nulls)}")

    # ablation: the same sweep without wave aggregation (one queue operation
    # per lane), one step
    ablation = None
    if not args.no_ablation:
        a = run_sweep(args.variant, 1, 1, count=False, width=1)
        ablation = {"width": 1, "variant": args.variant, "value": a["value"],
                    "value_all_iterations": a["value_all_iterations"],
                    "per_size_ops_per_s": {k: v["ops_per_s"] for k, v in a["per_size"].items()},
                    "aggregation_speedup": head["value"] / a["value"]}
        log(f"width 1 ablation: {a['value']/1e9:.2f} G ops/s")


    # ---------------- plain baseline: runtime device malloc/free ----------------
    # the same driver loop as ours (alloc -> write -> check -> free, ten
    # iterations per size, 2^20 threads at every size); requests the runtime
    # cannot serve come back NULL and are counted, never shrunk away.  Sizes
    # above 2 KiB are left out of the default run (its per-thread allocator
    # needs 44 s per iteration at 4 KiB) and are named as not run.
    plain = None
    if not args.no_plain:
        plain_sizes = [s for s in (int(x) for x in args.plain_sizes.split(",")) if s in sizes_list]
        plain = {"sizes": {}, "threads": n, "iterations": args.plain_iters,
                 "not_run": [s for s in sizes_list if s not in plain_sizes]}
        plain["heap_limit_rc"] = hb.hb_plain_set_heap(6 << 30)
        plain["heap_limit_bytes"] = 6 << 30
        p_ptrs = torch.zeros(n, dtype=torch.int64, device=dev)
        p_mism = torch.zeros(1, dtype=torch.int64, device=dev)
        tot_ops = tot_t = 0.0
        nulls = 0
        for s in plain_sizes:
            sd = size_dev[s]
            ta, tf, oks = [], [], []
            mism0 = int(p_mism.item())
            for it in range(args.plain_iters):
                e = [ev() for _ in range(4)]
                e[0].record()
                hb.hb_plain_alloc(sd, p_ptrs)
                e[1].record()
                hb.hb_plain_pattern(p_ptrs, sd, w.seed)
                hb.hb_plain_pattern(p_ptrs, sd, w.seed, p_mism)
                ok = int((p_ptrs != 0).sum().item())
                e[2].record()
                hb.hb_plain_free(p_ptrs)
                e[3].record()
                torch.cuda.synchronize()
                ta.append(e[0].elapsed_time(e[1]) / 1e3)
                tf.append(e[2].elapsed_time(e[3]) / 1e3)
                oks.append(ok)
                log(f"plain size={s} iteration {it + 1}: ok {ok} of {n}, alloc {ta[-1]*1e3:.1f} ms, "
                    f"free {tf[-1]*1e3:.1f} ms")
            sub = slice(1, None) if len(ta) > 1 else slice(0, None)
            t_sub = sum(ta[sub]) + sum(tf[sub])
            ops_sub = 2 * sum(oks[sub])
            nulls += sum(n - x for x in oks)
            plain["sizes"][str(s)] = {"ok_per_iteration": oks, "mismatched_words": int(p_mism.item()) - mism0,
                                      "alloc_us": [round(x * 1e6, 1) for x in ta],
                                      "free_us": [round(x * 1e6, 1) for x in tf],
                                      "ops_per_s_subsequent": ops_sub / t_sub if t_sub else None}
            tot_ops += ops_sub
            tot_t += t_sub
        plain["null_requests"] = nulls
        plain["mismatches"] = int(p_mism.item())
        plain["value"] = tot_ops / tot_t if tot_t else None
        # ours over the same sizes and iterations (2..10 of each size)
        o_ops = o_t = 0.0
        for s in plain_sizes:
            v = head["per_size"][str(s)]
            o_ops += 2 * v["ok"]
            o_t += (v["alloc_us"] + v["free_us"]) * 1e-6
        plain["ours_same_sizes"] = o_ops / o_t if o_t else None

    # ---------------- CPU baseline: the oracle on a bounded sample ----------------
    cpu = None
    if not args.no_cpu:
        import oracle as O
        O.build(force=False)
        variant = VARIANTS[args.variant]
        t_cpu, cpu_ops, passes = 0.0, 0, 0
        while t_cpu < args.cpu_seconds and passes < 50:
            h = O.OracleHeap(w.heap_bytes, w.chunk_bytes, variant)
            for s in sizes_list:
                sz = inputs.sizes_fixed(n, s)
                c0 = time.perf_counter()
                offs = h.alloc_batch(sz)
                h.free_batch(offs)
                h.trim()
                t_cpu += time.perf_counter() - c0
                cpu_ops += 2 * int((offs >= 0).sum())
            h.close()
            passes += 1
        cpu = {"value": cpu_ops / t_cpu, "unit": "ops/s", "cores": 1, "kind": "oracle",
               "sample": f"{passes} pass(es) of the sweep ({len(sizes_list)} sizes x 2^20 alloc+free, trim "
                         f"between sizes) through the sequential oracle, {t_cpu:.1f} s",
               "cpu_model": _cpu_model(), "host_cores_available": os.cpu_count()}

    # ---------------- context: the host C library's malloc/free, all host threads ----------------
    host_malloc = None
    if not args.no_host_malloc:
        threads = max(1, min(16, os.cpu_count() or 1))
        iters = max(2, args.host_malloc_iters)
        secs, failed = hb.hb_host_malloc_sweep(sizes_list, n, iters, threads)
        later = secs[:, 1:]
        host_malloc = {
            "value": 2.0 * n * later.size / float(later.sum()),
            "unit": "ops/s",
            "threads": threads,
            "kind": "host C library malloc/free",
            "sample": f"{len(sizes_list)} sizes x {iters} rounds of 2^20 malloc then 2^20 free split over "
                      f"{threads} threads; value over rounds 2..{iters}",
            "per_size_ops_per_s": {str(sz): 2.0 * n * (iters - 1) / float(later[i].sum())
                                   for i, sz in enumerate(sizes_list)},
            "failed": failed,
            "cpu_model": _cpu_model(),
            "host_cores_available": os.cpu_count(),
        }
        log(f"host malloc/free: {host_malloc['value'] / 1e6:.1f} M ops/s on {threads} threads")

    paper = None if args.no_paper_sweeps else bench_paper_sweeps(hb, inputs, torch, args, ev, log)
    growth = None if args.no_growth else bench_growth(hb, inputs, torch, args, ev, log)
    serve = None if args.no_serve else bench_serve(hb, inputs, torch, args, log)

    detail = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "fixed-size sweep: 4 GiB heap, 8 KiB chunks, 2^20 threads per launch, one size per launch "
                        "16 B..8 KiB, 10 x (alloc -> write -> check -> free) per size, trim between sizes; value over "
                        "iterations 2..10",
            "variant": args.variant,
            "aggregation_width": args.width,
            "shards": head["shards"],
            "iterations_per_size": args.iters,
            "requests_per_lane": args.rows or 4,
            "sizes": sizes_list,
        },
        "headline": head,
        "ceilings_g_per_s": {k: v / 1e9 for k, v in ceilings.items()},
        "latency_chain_us": {str(FAST_PATH_ROUND_TRIPS): chain_us, "1": chain1_us},
        "copy_gb_per_s": copy_gbps,
        "event_overhead_us": ev_overhead,
        "other_variant": other,
        "va_variant": va,
        "va_chunk_variant": va_chunk,
        "vl_variant": virt.get("vl-page"),
        "vl_chunk_variant": virt.get("vl-chunk"),
        "eager_chunk_variant": eager,
        "ablation_width1": ablation,
        "plain": plain,
        "vs_plain": (plain["ours_same_sizes"] / plain["value"])
        if plain and plain["value"] and plain["ours_same_sizes"] else None,
        "cpu_baseline": cpu,
        "host_malloc_context": host_malloc,
        "paper_sweeps": paper,
        "growth": growth,
        "serving": serve,
        "detail_path": args.detail or None,
    }
    text = json.dumps(detail)
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            f.write(text + "\n")
    else:
        print("detail " + text, file=sys.stderr, flush=True)
    print(json.dumps(compact(detail)), flush=True)


def bench_paper_sweeps(hb, inputs, torch, args, ev, log):
    """The paper's driver loop (Methods) on its two sweeps (Results): 1024
    allocations at each size 16 B .. 8 KiB, and 1 .. 2^20 threads allocating
    1000 B.  Ten iterations of allocate -> write -> check -> free on a 4 GiB
    heap of 8 KiB chunks; reported: the mean allocation and free launch time
    over all iterations and over iterations 2..10 (the paper's "subsequent
    iterations")."""
    import numpy as np
    w = inputs.SWEEP

    def point(heap, n, size):
        sd = torch.from_numpy(inputs.sizes_fixed(n, size).view(np.int64)).to("cuda")
        ptrs = torch.zeros(n, dtype=torch.int64, device="cuda")
        mism = torch.zeros(1, dtype=torch.int64, device="cuda")
        ta, tf = [], []
        hold_stream(torch)
        evs = []
        for it in range(10):
            e = [ev() for _ in range(4)]
            e[0].record()
            heap.alloc(sd, ptrs)
            e[1].record()
            hb.heap_pattern_write(heap.h, ptrs, sd, w.seed)
            hb.heap_pattern_check(heap.h, ptrs, sd, w.seed, mism)
            e[2].record()
            heap.free(ptrs)
            e[3].record()
            evs.append(e)
        torch.cuda.synchronize()
        for e in evs:
            ta.append(e[0].elapsed_time(e[1]) * 1e3)
            tf.append(e[2].elapsed_time(e[3]) * 1e3)
        heap.trim()
        assert int(mism.item()) == 0
        return {"alloc_us_all": float(np.mean(ta)), "alloc_us_subsequent": float(np.mean(ta[1:])),
                "free_us_all": float(np.mean(tf)), "free_us_subsequent": float(np.mean(tf[1:]))}

    res = {"workload": "4 GiB heap, 8 KiB chunks; 10 x (alloc -> write -> check -> free) per point",
           "size_sweep_1024_allocs": {}, "thread_sweep_1000B": {}}
    for vname, variant in (("chunk", hb.VARIANT_CHUNK), ("page", hb.VARIANT_PAGE), ("va-page", hb.VARIANT_VA_PAGE),
                           ("va-chunk", hb.VARIANT_VA_CHUNK), ("vl-page", hb.VARIANT_VL_PAGE),
                           ("vl-chunk", hb.VARIANT_VL_CHUNK)):
        with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant) as heap:
            res["size_sweep_1024_allocs"][vname] = {
                str(s_): point(heap, inputs.PAPER_ALLOCS, s_) for s_ in inputs.SWEEP_SIZES}
            res["thread_sweep_1000B"][vname] = {
                str(t): point(heap, t, inputs.PAPER_SIZE) for t in inputs.PAPER_THREADS}
            assert heap.error() == 0
    ts = res["thread_sweep_1000B"]["page"]
    log("paper sweeps: page, 1000 B: " + ", ".join(f"{t}: {v['alloc_us_subsequent']:.1f} us"
                                                    for t, v in ts.items()))
    return res


def bench_growth(hb, inputs, torch, args, ev, log):
    """Growth line: 2^18 agents on a 4 GiB heap grow int32 lists 16 B ->
    4 KiB over nine steps (dev_malloc / copy / dev_free per doubling).  The
    autotuner picks (chunk size, variant, width) on one seeded schedule; the
    pick and the default are then timed on another (graph replays, median)."""
    import numpy as np
    w = inputs.GROWTH
    agents, steps = w.threads, w.rounds
    KiB = 1024
    d_cal = inputs.growth_doublings(agents, w.seed * 16 + 0xA)   # 0xC0F4A
    d_eval = inputs.growth_doublings(agents, w.seed * 16 + 0xB)  # 0xC0F4B
    cands = [(c * KiB, v, wd, 0) for c in (8, 16, 32, 64) for v in (0, 1, 2, 3, 4, 5) for wd in (16, 32, 64)]
    # the chunk variant with eager retirement
    cands += [(c * KiB, hb.VARIANT_CHUNK, wd, hb.FLAG_EAGER) for c in (8, 16, 32, 64) for wd in (16, 32, 64)]
    t0 = time.perf_counter()
    ms, best = hb.growth_autotune(w.heap_bytes, agents, torch.from_numpy(d_cal).to("cuda"), steps, w.seed, cands,
                                  reps=5)
    tune_s = time.perf_counter() - t0
    if best < 0:
        log("growth autotuner: no candidate ran")
        return {"error": "no candidate ran"}
    default = (8 * KiB, 1, 64, 0)

    def cname(cfg):
        c, v, wd, fl = cfg
        return f"{c // KiB}K/{VNAMES[v]}{'-eager' if fl else ''}/w{wd}"

    def measure(cfg, d):
        chunk, variant, width, flags = cfg
        with hb.Heap(w.heap_bytes, chunk, variant=variant, width=width, flags=flags) as heap:
            with hb.Growth(heap, torch.from_numpy(d).to("cuda"), steps, w.seed) as gr:
                gr.run_graph()
                gr.release()
                graph_t, step_t = [], []
                for _ in range(args.growth_reps):
                    e0, e1 = ev(), ev()
                    e0.record()
                    gr.run_graph()
                    e1.record()
                    _, nbytes, fails = gr.export()
                    gr.release()
                    torch.cuda.synchronize()
                    assert fails == 0
                    graph_t.append(e0.elapsed_time(e1))
                for _ in range(5):
                    e0, e1 = ev(), ev()
                    e0.record()
                    for s_ in range(steps):
                        gr.step(s_)
                    e1.record()
                    gr.release()
                    torch.cuda.synchronize()
                    step_t.append(e0.elapsed_time(e1))
                final_bytes = int(nbytes.sum().item())
                blocks, threads = gr.shape()
            assert heap.error() == 0
        return float(np.median(graph_t)), float(np.median(step_t)), final_bytes, blocks * threads

    # per replay: step 0 allocates for every agent; each doubling allocates,
    # copies the old list and frees it
    doublings = int(d_eval.sum())
    reallocs = agents + doublings
    copied = int(sum((16 << s_) // 2 * int((d_eval >= s_).sum()) for s_ in range(1, steps)))
    written = int(sum((16 << s_) * int((d_eval >= s_).sum()) for s_ in range(1, steps))) + 16 * agents
    g_best, e_best, fb, lanes = measure(cands[best], d_eval)
    g_def, e_def, _, _ = measure(default, d_eval)
    res = {
        "workload": f"{agents} agents, 4 GiB heap, {steps} steps (16 B -> 4 KiB doubling reallocs), "
                    "doublings min(8, Geom(0.3)), calibration and evaluation schedules seeded apart",
        "graph_ms": g_best,
        "step_by_step_ms": e_best,
        "realloc_ops": reallocs,
        "alloc_free_ops_per_s": (reallocs + doublings) / (g_best * 1e-3),
        "payload_gb_per_s": (copied + written) / (g_best * 1e-3) / 1e9,
        "final_live_bytes": fb,
        "persistent_lanes": lanes,
        "autotune": {
            "best": {"chunk_bytes": cands[best][0], "variant": VNAMES[cands[best][1]],
                     "width": cands[best][2], "eager_retirement": bool(cands[best][3])},
            "calibration_ms": {cname(cf): round(t, 4) for cf, t in zip(cands, ms)},
            "default": {"chunk_bytes": default[0], "variant": "page", "width": default[2]},
            "default_graph_ms": g_def,
            "margin_vs_default": g_def / g_best,
            "seconds": tune_s,
        },
    }
    log(f"growth: graph {g_best:.3f} ms (step by step {e_best:.3f} ms), {res['alloc_free_ops_per_s']/1e9:.2f} G ops/s, "
        f"autotune best {res['autotune']['best']} margin {g_def / g_best:.3f}")
    return res


def bench_serve(hb, inputs, torch, args, log):
    """Serving line: 16 GiB heap (page variant), K slot streams, batches of
    mean 4096 requests (64..65536) with sizes log-uniform in [16 B, 8 KiB];
    warm-up to about half the heap, then mixed allocations and frees.  The
    capacity run offers every batch at once; then Poisson arrivals at 0.25,
    0.5 and 0.9 of that capacity."""
    import numpy as np
    w = inputs.SERVE
    mean_block = 1817  # mean class size of log-uniform [16, 8192]
    warm_req = int(0.5 * w.heap_bytes / mean_block)
    t0 = time.perf_counter()
    # enough batches for the warm-up plus the mixed phase
    est_warm = int(warm_req / 4096 * 1.1) + 16
    plan = inputs.serve_plan(est_warm + args.serve_batches, w.seed, warm_requests=warm_req)
    gen_s = time.perf_counter() - t0
    log(f"serving: plan of {len(plan.first) - 1} batches ({len(plan.ops)} requests) in {gen_s:.1f} s")
    nb = len(plan.first) - 1
    wb = plan.warm_batches
    mixed = slice(wb, nb)
    mixed_req = int(plan.first[nb] - plan.first[wb])

    def run(arr):
        with hb.Heap(w.heap_bytes, w.chunk_bytes, variant=hb.VARIANT_PAGE) as heap:
            s = hb.serve_create(heap.h, args.serve_slots, int(np.diff(plan.first).max()), len(plan.ops), 0.95,
                                w.seed, plan.free_lag)
            try:
                r = hb.serve_run(s, plan.first, plan.ops, arr, alone=False)
            finally:
                hb.serve_destroy(s)
            assert heap.error() == 0
        bad = int((r["status"] != 0).sum())
        lat = r["latency_ns"][mixed] / 1e3
        wait = r["wait_ns"][mixed] / 1e3
        # mixed phase: from the later of its first arrival and the end of the
        # warm-up, to its last completion
        done_ns = arr + r["latency_ns"]
        warm_done = float(np.max(done_ns[:wb])) * 1e-9 if wb else 0.0
        t_end = float(np.max(done_ns[mixed])) * 1e-9
        t_beg = max(float(arr[wb]) * 1e-9, warm_done)
        span = max(t_end - t_beg, 1e-9)
        return {"served_ops_per_s": mixed_req / span, "batches_per_s": (nb - wb) / span, "warm_done_s": warm_done,
                "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "admission_wait_us": {"p50": float(np.percentile(wait, 50)), "p99": float(np.percentile(wait, 99))},
                "failed_requests": bad, "trims": r["stats"]["trims"],
                "admission_stalls": r["stats"]["admission_stalls"], "peak_chunk_bound": r["stats"]["peak_bound"]}

    # capacity: warm-up and mixed batches all offered at time 0
    cap = run(np.zeros(nb, dtype=np.uint64))
    rate_cap = cap["batches_per_s"]
    log(f"serving: capacity {rate_cap:.0f} batches/s")
    points = {"capacity": cap}
    # load points: the warm-up is offered at time 0, the mixed batches arrive
    # (Poisson) from a little after the capacity run's warm-up ended
    start_ns = int(cap["warm_done_s"] * 1.25e9)
    for f in (0.25, 0.5, 0.9):
        arr = np.zeros(nb, dtype=np.uint64)
        arr[wb:] = inputs.arrivals_ns(nb - wb, f * rate_cap, w.seed + int(f * 100)) + np.uint64(start_ns)
        points[f"load_{f}"] = run(arr)
        log(f"serving load {f}: p50 {points[f'load_{f}']['latency_us']['p50']:.1f} us, "
            f"p99 {points[f'load_{f}']['latency_us']['p99']:.1f} us")
    res = {
        "workload": f"16 GiB heap, page variant, {args.serve_slots} slot streams, admission at 95% of chunks; "
                    f"{wb} warm-up batches ({int(plan.first[wb])} allocations), then {nb - wb} mixed batches "
                    f"({mixed_req} requests, half frees) per load point",
        "capacity_batches_per_s": rate_cap,
        "points": points,
        "plan_seconds": gen_s,
    }
    log(f"serving: capacity {rate_cap:.0f} batches/s, {cap['served_ops_per_s']/1e9:.3f} G ops/s")
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
