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
2..10 (HIP events on the launch stream); iterations 1..10 are reported too.
Each size's ten iterations are queued behind a short device-side wait, so
every event pair times its launch on the device's timeline rather than the
host's submission latency.  The whole step's wall time (payload write/check,
those waits and trims included) is ms_per_step, and all ops over it is
wall_ops_per_s.

The headline runs the page-queue variant (the faster one on this workload);
the chunk-queue variant runs the same sweep for one step beside it.

Also measured in the same process:
  * the device atomic ceilings (same address, 64 and 1024 lines, per-lane
    random addresses);
  * a counting pass with the heap's statistics flag, giving the exact
    atomics issued per launch by target; the roofline compares all atomics
    of the allocation launch per second with the measured device atomic
    throughput, and the busiest queue word with the same-address ceiling;
  * the plain baseline: the runtime's own per-thread device malloc/free;
  * the CPU baseline: the sequential oracle on a bounded sample, one core.

roofline.traffic is the HBM bytes per allocation launch (FETCH_SIZE and
WRITE_SIZE counters, scaled by the same counters' reading for a copy of known
size) recorded in the counter summary under profiles/; it is null once the
kernel sources differ from the digest stored there.

Prints one JSON line.  Only --gpus 1 is supported.  `--copy-probe BYTES`
only runs the HBM copy kernel (to calibrate traffic counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=10, help="alloc-write-check-free iterations per size")
    ap.add_argument("--variant", choices=["chunk", "page", "va-page", "va-chunk", "vl-page", "vl-chunk"],
                    default="page")
    ap.add_argument("--width", type=int, default=64)
    ap.add_argument("--shards", type=int, default=0, help="queue shards (0: one per 256 chunks, up to 64)")
    ap.add_argument("--no-other", action="store_true", help="skip the other queue variant")
    ap.add_argument("--no-va", action="store_true", help="skip the virtualised-array and -list variant lines")
    ap.add_argument("--no-eager", action="store_true", help="skip the eager chunk retirement line")
    ap.add_argument("--no-ablation", action="store_true", help="skip the width-1 (no aggregation) ablation")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain device-malloc baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--sizes", type=str, default="", help="comma list overriding the 16..8192 sweep")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run an HBM copy of this many bytes")
    ap.add_argument("--no-growth", action="store_true", help="skip the growth line (graph replay, autotuner)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving line")
    ap.add_argument("--no-paper-sweeps", action="store_true", help="skip the paper's size and thread sweeps")
    ap.add_argument("--growth-reps", type=int, default=20)
    ap.add_argument("--serve-batches", type=int, default=10000, help="mixed batches per load point")
    ap.add_argument("--serve-slots", type=int, default=4)
    return ap.parse_args()


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

    # ---------------- atomic ceilings ----------------
    def probe(pattern, lines, threads, iters):
        buf = torch.zeros(64 << 20, dtype=torch.uint8, device=dev)
        best = None
        for _ in range(3):
            e0, e1 = ev(), ev()
            e0.record()
            hb.hb_atomic_probe(pattern, buf, buf.numel(), threads, lines, iters)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / 1e3
            best = t if best is None else min(best, t)
        n_at = threads * iters if pattern in (2, 4, 5, 6, 7) else threads // 64 * iters
        return n_at / best

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
    ceil_same = probe(0, 1, 1 << 20, 4)
    ceil_64 = probe(1, 64, 1 << 20, 4)
    ceil_lines = probe(1, 1024, 1 << 20, 4)
    ceil_spread = probe(2, 1, 1 << 20, 4)
    log(f"atomic ceilings: same-address {ceil_same/1e9:.3f} G/s, 64 lines {ceil_64/1e9:.2f} G/s, "
        f"1024 lines {ceil_lines/1e9:.2f} G/s, per-lane random {ceil_spread/1e9:.2f} G/s")

    size_dev = {s: torch.from_numpy(inputs.sizes_fixed(n, s).view(np.int64)).to(dev) for s in sizes_list}
    ptrs = torch.zeros(n, dtype=torch.int64, device=dev)
    mism = torch.zeros(1, dtype=torch.int64, device=dev)
    keys = ("state_ops", "headtail_ops", "pool_ops", "spread_ops")

    def run_sweep(variant_name: str, steps: int, warmup: int, count: bool, width: int | None = None) -> dict:
        variant = VARIANTS[variant_name]
        heap = hb.Heap(w.heap_bytes, w.chunk_bytes, variant=variant, width=args.width if width is None else width,
                       shards=args.shards, flags=CREATE_FLAGS.get(variant_name, 0))
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

        per_size = {s: {"alloc_us": [], "free_us": [], "ok": 0} for s in sizes_list}
        sub_ops = sub_t = all_ops = all_t = 0.0
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
            per_size[s]["ok"] = okv
        out = {
            "variant": variant_name,
            "shards": shards,
            "value": sub_ops / sub_t,
            "value_all_iterations": all_ops / all_t,
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
            # roofline of the dominant kernel, k_alloc_batch: all atomics it
            # issues (counted in the counting pass) per launch over the average
            # time of every non-counting allocation launch of this sweep
            # (warmup + timed: the population a kernel trace averages over),
            # against the measured device atomic throughput; the busiest queue
            # word (a class state word, spread over the shards) against the
            # same-address ceiling
            alloc_t, atomics, state_atomics = [], 0, 0
            for s, it, e, ok in warm + recs:
                alloc_t.append(e[0].elapsed_time(e[1]) / 1e3)
                cnt = counts[s]["first" if it == 0 else "subsequent"]["alloc"]
                atomics += sum(cnt.values())
                state_atomics += cnt["state_ops"]
            t_sum = sum(alloc_t)
            achieved = atomics / t_sum
            busiest = state_atomics / shards / t_sum
            out["roofline"] = {
                "bound": "atomic",
                "kernel": f"k_alloc_batch<false, {variant}u>",
                "achieved": achieved / 1e9,
                "peak": ceil_spread / 1e9,
                "unit": "Gatomic/s (device-scope atomics issued; peak = measured per-lane random atomic throughput)",
                "frac": achieved / ceil_spread,
                "traffic": recorded_traffic(),
                "avg_launch_us": float(np.mean(alloc_t)) * 1e6,
                "event_overhead_us": ev_overhead,
                "launches": len(alloc_t),
                "atomics_per_launch": atomics / len(alloc_t),
                "busiest_word": {"achieved": busiest / 1e9, "peak": ceil_same / 1e9, "frac": busiest / ceil_same,
                                 "state_word_atomics_per_launch": state_atomics / len(alloc_t), "shards": shards},
                "alloc_share_of_alloc_free_time": sum(t_alloc_sub) / (sum(t_alloc_sub) + sum(t_free_sub)),
            }
        return out

    head = run_sweep(args.variant, args.steps, args.warmup, count=True)
    log(f"{args.variant}: {head['value']/1e9:.2f} G ops/s (iterations 2..10)")
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
        log(f"chunk-eager: {eager['value']/1e9:.2f} G ops/s (iterations 2..10), roofline frac "
            f"{eager['roofline']['frac']:.3f} ({eager['roofline']['atomics_per_launch']:.0f} atomics per launch)")
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
    plain = None
    if not args.no_plain:
        plain = {"sizes": {}}
        rc = hb.hb_plain_set_heap(6 << 30)
        plain["heap_limit_rc"] = rc
        p_ptrs = torch.zeros(n, dtype=torch.int64, device=dev)
        tot_ops, tot_t = 0, 0.0
        for s in sizes_list:
            nn = n if s <= 1024 else (1 << 16)
            sd = size_dev[s][:nn]
            pp = p_ptrs[:nn]
            e = [ev() for _ in range(4)]
            e[0].record()
            hb.hb_plain_alloc(sd, pp)
            e[1].record()
            ok = int((pp != 0).sum().item())
            e[2].record()
            hb.hb_plain_free(pp)
            e[3].record()
            torch.cuda.synchronize()
            t = (e[0].elapsed_time(e[1]) + e[2].elapsed_time(e[3])) / 1e3
            plain["sizes"][str(s)] = {"threads": nn, "ok": ok, "ops_per_s": round(2 * ok / t, 0),
                                      "alloc_us": round(e[0].elapsed_time(e[1]) * 1e3, 1),
                                      "free_us": round(e[2].elapsed_time(e[3]) * 1e3, 1)}
            if nn == n:
                tot_ops += 2 * ok
                tot_t += t
            log(f"plain size={s} threads={nn} ok={ok} {2*ok/t/1e6:.2f} M ops/s")
        plain["value_full_size_sizes"] = tot_ops / tot_t if tot_t else None
        # ours over the same sizes (those the plain kernel ran at 2^20 threads)
        o_ops = o_t = 0.0
        for s in sizes_list:
            if s <= 1024:
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

    paper = None if args.no_paper_sweeps else bench_paper_sweeps(hb, inputs, torch, args, ev, log)
    growth = None if args.no_growth else bench_growth(hb, inputs, torch, args, ev, log)
    serve = None if args.no_serve else bench_serve(hb, inputs, torch, args, log)

    out = {
        "metric": "device malloc+free ops/sec (2^20 threads, 16B-8KiB) vs plain; p99 batch latency",
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
            "sizes": sizes_list,
        },
        "value_all_iterations": head["value_all_iterations"],
        "wall_ops_per_s": head["wall_ops_per_s"],
        "batch_latency_us": head["batch_latency_us"],
        "roofline": head["roofline"],
        "atomic_ceilings_gps": {"same_address": ceil_same / 1e9, "lines_64": ceil_64 / 1e9,
                                "lines_1024": ceil_lines / 1e9, "per_lane_random": ceil_spread / 1e9},
        "per_size": head["per_size"],
        "other_variant": other,
        "va_variant": va,
        "va_chunk_variant": va_chunk,
        "vl_variant": virt.get("vl-page"),
        "vl_chunk_variant": virt.get("vl-chunk"),
        "eager_chunk_variant": eager,
        "ablation_width1": ablation,
        "plain": plain,
        "vs_plain": (plain["ours_same_sizes"] / plain["value_full_size_sizes"])
        if plain and plain["value_full_size_sizes"] and plain["ours_same_sizes"] else None,
        "cpu_baseline": cpu,
        "paper_sweeps": paper,
        "growth": growth,
        "serving": serve,
    }
    print(json.dumps(out), flush=True)


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
