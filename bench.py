#!/usr/bin/env python3
"""Throughput of BMMC permutations on one MI355X.

Default workload: a uniformly random invertible 26 x 26 matrix over F_2 with a
random complement (seed 0), applied to 2^26 int32 elements drawn from seed 0.
The timed path is the library's default call with autotuned options: one
LDS-staged pass over the HBM-resident array (a general tile; tiled matrices
take the paper's tiled pass), unless the tuner found the paper's two tiled
passes faster.  One step is one whole permutation.  The paper's two-pass
scheme (Section 5.2) on the same input is timed beside it.

Prints ONE JSON line.  `value` is effective throughput in GB/s (decimal):
algorithmic bytes (one read plus one write of the array, 2 * 2^n * w) per step
time.  Beside it: the best same-session device copy and the HBM peak as
fractions, the roofline of the dominant kernel, the paper's two-pass scheme,
the naive lower bound, the batched form (1024 arrays, one graph launch,
against 1024 separate calls; p50/p99 of the batch latency), the served form
(Poisson arrivals at 20k requests/s and, past the server's capacity, at 60k;
p50/p99 request latency beside the same requests as per-request launches)
and the CPU oracle's rate on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BMMC permute GB/s (rd+wr) as % of device copy & HBM peak; batched p99 latency"
# Autotuner results for this GPU (JSON lines of the library's tuning cache,
# which the library also loads by itself): used unless --retune; --save-tune
# writes a run's results in the same form.
TUNE_DB = os.path.join(ROOT, "paper_2306_07795_amd", "tuning", "gfx950.jsonl")
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    # name: (n, elem_bytes, matrix kind, description)
    "random26": (26, 4, "random", "random BMMC on 2^26 int32 (A uniform invertible 26x26 over F_2, "
                                  "random c, seed 0)"),
    "random28": (28, 4, "random", "random BMMC on 2^28 int32 (seed 0)"),
    "random27x8": (27, 8, "random", "random BMMC on 2^27 int64 (seed 0)"),
    "bitrev28": (28, 4, "bitrev", "bit reversal of 2^28 int32"),
    "bitrev27x8": (27, 8, "bitrev", "bit reversal of 2^27 int64"),
    "swap28": (28, 4, "swap", "2^14 x 2^14 int32 matrix transpose (bit-block swap)"),
    "swap27x8": (27, 8, "swap", "2^13 x 2^14 int64 matrix transpose (bit-block swap)"),
    "bitrev20": (20, 4, "bitrev", "bit reversal of 2^20 int32 (cache resident)"),
    "reverse27": (27, 4, "reverse", "reversal x -> x XOR (2^27 - 1) of 2^27 int32 (identity matrix, all-ones c)"),
}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "pass.hpp"):
        with open(os.path.join(ROOT, "paper_2306_07795_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def matrix(kind, n, seed=0):
    from synth import gen
    if kind == "random":
        return gen.random_bmmc(n, seed)
    if kind == "bitrev":
        return gen.bit_reversal_rows(n), 0
    if kind == "swap":
        return gen.block_swap_rows(n, n // 2), 0
    if kind == "reverse":
        return gen.identity_rows(n), (1 << n) - 1
    raise ValueError(kind)


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def gbps(nbytes, ms):
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def progress(msg):
    """One line on stderr as each part of a run finishes."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


# Cache state of the headline: before every timed call, a copy of
# FLUSH_BYTES between two other buffers (outside the timed interval) leaves
# the L2 caches and the 256 MB last-level cache holding another array's
# lines, many of them dirty -- the state of a call that follows unrelated
# work.  The library's autotuner times calls of 64 MiB and more the same way.
FLUSH_BYTES = 512 << 20
FLUSH_KERNEL = "k_copy<1,0>"


class Flusher:
    def __init__(self, device):
        import torch
        self.a = torch.full((FLUSH_BYTES,), 0x3C, dtype=torch.uint8, device=device)
        self.b = torch.empty_like(self.a)

    def __call__(self, stream):
        from paper_2306_07795_amd import binding as B
        B.bmmc_copy_ex(self.a, self.b, FLUSH_BYTES, 1, 0, stream)


def flushed_times(fn, reps, warmup, stream, flush):
    """Per-call times (ms) of fn(), each call right after a cache flush; HIP
    events on the stream around the call only."""
    import torch
    for _ in range(warmup):
        flush(stream)
        fn()
    evs = []
    for _ in range(reps):
        flush(stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        evs.append((a, b))
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def mean(v):
    return sum(v) / len(v)


def profiled_kernels(fn, reps, stream, flush):
    """(name, stats) of the dominant kernel over `reps` calls of fn, each
    after a cache flush, with the library's kernel-bound events on.  Kept
    apart from the timed calls: the profiling bookkeeping lengthens a call
    by several microseconds."""
    import torch
    from paper_2306_07795_amd import binding as B
    B.bmmc_profile_begin()
    for _ in range(reps):
        flush(stream)
        fn()
    torch.cuda.synchronize()
    return dominant(B.bmmc_profile_end())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(a, n, rows, c, run_s=4.0, runs=3):
    """The oracle, as is, on this host's cores: `runs` runs, each repeating
    the full workload until about run_s seconds have passed (at least once);
    the median run's rate is the value.  Then one run on a single thread."""
    from oracle import oracle as orc
    cores = orc.threads(0)
    rates, reps_per_run = [], []
    for _ in range(runs):
        reps, t0 = 0, time.perf_counter()
        while True:
            orc.permute(a, n, rows, c, 0)
            reps += 1
            if time.perf_counter() - t0 > run_s or reps >= 200:
                break
        dt = (time.perf_counter() - t0) / reps
        rates.append(2.0 * a.nbytes / dt / 1e9)
        reps_per_run.append(reps)
    med = sorted(rates)[len(rates) // 2]
    t1 = time.perf_counter()
    orc.permute(a, n, rows, c, 1)
    dt1 = time.perf_counter() - t1
    return {"value": round(med, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(), "runs_GBps": [round(r, 3) for r in rates],
            "value_1_thread": round(2.0 * a.nbytes / dt1 / 1e9, 3),
            "sample": f"the full workload (2^{n} elements), median of {runs} runs of about {run_s:.0f} s "
                      f"({'/'.join(map(str, reps_per_run))} repetitions) on {cores} threads, then one of "
                      f"{dt1:.2f} s on 1 thread"}


def kernel_key(name):
    """'void bmmc::k_tiled<4, 256, 4, 3>(...)' -> 'k_tiled<4,256,4,3>'."""
    base = name.split("(")[0].replace("void ", "").replace("bmmc::", "")
    return base.replace(" ", "")


def write_traffic(fetch_dir, write_dir, nbytes, workload):
    """profiles/traffic.json, entry `workload`, from two rocprofv3 --pmc runs
    of this benchmark on that workload (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch).  Each counter is scaled by the ratio (algorithmic bytes /
    counter bytes) it shows for the plain copy kernel k_copy<4,0>, which
    reads and writes `nbytes` per launch.  Entries of other workloads are
    kept while the kernel source is unchanged."""
    import csv
    import glob
    import statistics

    def means(d, counter):
        out = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    out.setdefault(kernel_key(r["Kernel_Name"]), []).append(float(r["Counter_Value"]) * 1024.0)
        return {k: statistics.mean(v) for k, v in out.items()}

    fetch, write = means(fetch_dir, "FETCH_SIZE"), means(write_dir, "WRITE_SIZE")
    f_scale = nbytes / fetch["k_copy<4,0>"]
    w_scale = nbytes / write["k_copy<4,0>"]
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        rb, wb = fetch[k] * f_scale, write[k] * w_scale
        kernels[k] = {"read_bytes_per_launch": round(rb), "write_bytes_per_launch": round(wb),
                      "bytes_per_launch": round(rb + wb)}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    if rec.get("kernel_source_hash") != kernel_source_hash() or "workloads" not in rec:
        rec = {"kernel_source_hash": kernel_source_hash(), "workloads": {}}
    rec["workloads"][workload] = {"fetch_scale": f_scale, "write_scale": w_scale,
                                  "calibration": "k_copy<4,0> moving %d bytes each way" % nbytes,
                                  "kernels": kernels}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def traffic_for(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` measured with rocprofv3
    counters, if they were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = rec.get("workloads", {}).get(workload, {}).get("kernels", {}).get(kernel)
    return ent.get("bytes_per_launch") if ent else None


def best_device_copy(x, y, nbytes, stream, flush=None, reps=10):
    """Fastest of the copy kernel's variants and hipMemcpy (device to device):
    back to back (flush None), or each call after a cache flush."""
    from paper_2306_07795_amd import binding as B

    def t(fn):
        if flush is None:
            return timed(fn, reps, 2, stream)
        return mean(flushed_times(fn, reps, 2, stream, flush))
    best = (1e30, None)
    for vpt in (1, 2, 4, 8):
        for hints in (0, 1, 2, 3):
            ms = t(lambda: B.bmmc_copy_ex(x, y, nbytes, vpt, hints, stream))
            best = min(best, (ms, f"k_copy vpt={vpt} hints={hints}"))
    ms = t(lambda: y.copy_(x))
    best = min(best, (ms, "hipMemcpy device to device"))
    return best


def dominant(kstats):
    """(name, stats) of the kernel with the most time, flush copies excluded."""
    ks = {k: v for k, v in kstats.items() if k != FLUSH_KERNEL}
    return max(ks.items(), key=lambda kv: kv[1]["total_ms"])


def paper_two_pass(x, y, n, rows, c, w, stream, flush, copy_ms, warm_copy_ms, tune=True, retune=False):
    """The paper's scheme on the same input: the factorization into tiled
    BMMCs, two LDS-staged passes through scratch (Section 5.2), tuned the
    same way; each call after a cache flush (and back to back), with its
    dominant kernel's rate per launch (kernel-bound events)."""
    from paper_2306_07795_amd import binding as B
    nbytes = (1 << n) * w
    opts = {"method": B.METHOD_TILED}
    if tune:
        found = None if retune else B.bmmc_tune_lookup(n, w, rows, B.METHOD_TILED)
        if found is None:
            B.bmmc_autotune(n, w, B.METHOD_TILED, stream, 3)
            found = B.bmmc_tune_lookup(n, w, rows, B.METHOD_TILED)
        opts = found or opts
    passes = B.bmmc_plan_ex(rows, c, n, w, opts).nfactors
    call = lambda: B.bmmc_permute_ex(x, y, n, rows, c, w, opts, stream)  # noqa: E731
    ms = mean(flushed_times(call, 20, 3, stream, flush))
    kname, k = profiled_kernels(call, 10, stream, flush)
    warm_ms = timed(lambda: B.bmmc_permute_ex(x, y, n, rows, c, w, opts, stream), 20, 3, stream)
    v = gbps(nbytes, ms)
    per_launch = k["total_ms"] / k["launches"]
    return {"GBps": round(v, 1), "passes": passes, "pct_of_device_copy": round(100.0 * copy_ms / ms, 2),
            "traffic_pct_of_device_copy": round(100.0 * copy_ms * passes / ms, 2),
            "kernel": kname, "kernel_mean_launch_ms": round(per_launch, 5),
            "kernel_GBps": round(k["bytes"] / k["launches"] / (per_launch * 1e-3) / 1e9, 1),
            "warm": {"GBps": round(gbps(nbytes, warm_ms), 1),
                     "pct_of_device_copy": round(100.0 * warm_copy_ms / warm_ms, 2)},
            "options": opts}


def cache_states(x, y, n, rows, c, w, opts, two_pass_opts, stream, flush, reps=20):
    """The permutation and the copy bound in two other states than the
    headline's: "chained" alternates x -> m and m -> y, so that every call
    reads what the call before it has just written, as in a pipeline; and,
    after a cache flush like the headline, the timed options against
    non-temporal loads with cached stores (hints 1) and non-temporal loads
    and stores (hints 3).  Events around each call only; the copy is the
    fastest of its variants in the same state."""
    import torch
    from paper_2306_07795_amd import binding as B
    nbytes = (1 << n) * w
    m = torch.empty_like(x)

    def per_call(fns, before=None):
        evs = []
        for r in range(reps + 2):
            for fn in fns:
                if before:
                    before(stream)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                if r >= 2:
                    evs.append((a, b))
        torch.cuda.synchronize()
        return 1e3 * sum(a.elapsed_time(b) for a, b in evs) / len(evs)

    def perm(o):
        return [lambda: B.bmmc_permute_ex(x, m, n, rows, c, w, o, stream),
                lambda: B.bmmc_permute_ex(m, y, n, rows, c, w, o, stream)]

    variants = {"timed options": opts}
    if opts is not None:  # (None: the library's default call, whose options are its own)
        variants.update({"hints 1": dict(opts, hints=1), "hints 3": dict(opts, hints=3)})
    out = {}
    for state, before in (("chained", None), ("flushed", flush)):
        cp_us, cp_how = 1e30, None
        for vpt in (1, 2):
            for hints in (0, 1, 2, 3):
                t = per_call([lambda: B.bmmc_copy_ex(x, m, nbytes, vpt, hints, stream),
                              lambda: B.bmmc_copy_ex(m, y, nbytes, vpt, hints, stream)], before)
                cp_us, cp_how = min((cp_us, cp_how), (t, f"k_copy vpt={vpt} hints={hints}"))
        p_us = {k: per_call(perm(o), before) for k, o in variants.items()}
        t_us = per_call([lambda: B.bmmc_permute_ex(x, y, n, rows, c, w, two_pass_opts, stream)], before)
        out[state] = {"copy_us": round(cp_us, 1), "copy": cp_how,
                      "permute_us": {k: round(v, 1) for k, v in p_us.items()},
                      "pct_of_copy": {k: round(100.0 * cp_us / v, 1) for k, v in p_us.items()},
                      "paper_two_pass_us": round(t_us, 1),
                      "one_pass_speedup_vs_two": round(t_us / min(p_us.values()), 2)}
    del m
    return out


def other_matrices(x, y, n, w, copy_ms, stream, flush, seeds=8, reps=10):
    """The library's default call on random matrices of seeds 0..seeds-1 (the
    timed workload is seed 0), each call after a cache flush like the
    headline, then the same after tuning each matrix: beyond the last-level
    cache how the accesses meet the memory system varies from one matrix to
    another."""
    from paper_2306_07795_amd import binding as B
    from synth import gen
    pct, per = [], []
    for seed in range(seeds):
        rows, c = gen.random_bmmc(n, seed)
        ms = mean(flushed_times(lambda: B.bmmc_permute(x, y, n, rows, c, w, stream), reps, 2, stream, flush))
        pct.append(100.0 * copy_ms / ms)
    # the same calls after bmmc_autotune_matrix has tuned each matrix
    # (before the timed calls; the settings are dropped afterwards)
    try:
        for seed in range(seeds):
            rows, c = gen.random_bmmc(n, seed)
            B.bmmc_autotune_matrix(x, y, n, rows, c, w, stream, 3)
            ms = mean(flushed_times(lambda: B.bmmc_permute(x, y, n, rows, c, w, stream), reps, 2, stream, flush))
            per.append(100.0 * copy_ms / ms)
    finally:
        B.bmmc_tune_clear_matrices()

    def summary(v):
        return {"pct_of_device_copy": [round(p, 1) for p in v], "mean": round(sum(v) / len(v), 1),
                "min": round(min(v), 1), "max": round(max(v), 1)}
    return {"seeds": f"0-{seeds - 1}", "cache_state": "flushed", **summary(pct), "tuned_per_matrix": summary(per)}


def torch_sync():
    import torch
    torch.cuda.synchronize()


def bench_batched(count=1024, reps=50, seed=0, retune=False):
    """1024 arrays, n uniform in [10, 22], int32, each its own A and c: the
    resident batch (one graph replay of the persistent kernel) against the
    same 1024 arrays as separate bmmc_permute calls, both issued by the host
    (a ctypes loop) and captured once into a graph of 1024 launches and
    replayed (device time of separate launches, no host issue cost).  Batch
    latency = events around one launch or replay; p50/p99 over reps."""
    import ctypes

    import numpy as np
    import torch
    from paper_2306_07795_amd import binding as B
    from synth import gen
    sizes = gen.batched_sizes(count, seed, 10, 22)
    items, total = [], 0
    for k, n in enumerate(sizes):
        rows, c = gen.random_bmmc(n, 1_000_003 * (seed + 1) + k)
        x = torch.from_numpy(gen.data(n, 4, k).view(np.uint8)).to("cuda")
        y = torch.empty_like(x)
        items.append((x, y, n, 4, rows, c))
        total += (1 << n) * 4
    stream = torch.cuda.current_stream()
    tuned = None if retune else B.bmmc_tune_lookup_batched(items)
    if tuned is None:
        tuned, _ = B.bmmc_autotune_batched(items, stream, 2)

    def lat(fn, r):
        out = []
        for _ in range(r):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            out.append(a.elapsed_time(b))
        return np.array(out)

    # resident batch: one graph replay per launch (the descriptors, plans,
    # scratch and graph were made once)
    pb = B.bmmc_batch_create(items, tuned)
    pb.launch(stream)
    resident = lat(lambda: pb.launch(stream), reps)
    # one-shot batched call: the library's host work (plan lookups, table
    # fill and upload) included; the descriptors are marshalled once
    descs = B.DescBatch(items)
    oneshot = lat(lambda: B.bmmc_permute_batched(descs, stream, tuned), max(5, reps // 5))

    # 1024 separate library calls, their arguments marshalled once
    lib = B.lib()
    calls = [(ctypes.c_void_p(it[0].data_ptr()), ctypes.c_void_p(it[1].data_ptr()), it[2],
              (ctypes.c_uint64 * it[2])(*[int(v) for v in it[4]]), ctypes.c_uint64(it[5])) for it in items]

    def separate(s):
        sp = ctypes.c_void_p(s.cuda_stream)
        for i, o, n, r, c in calls:
            if lib.bmmc_permute(i, o, n, r, c, 4, sp) != 0:
                raise SystemExit("bmmc_permute failed: " + lib.bmmc_last_error().decode())

    sep = lat(lambda: separate(stream), max(5, reps // 5))
    # the same 1024 calls captured into one graph (plans made by the calls
    # above; one-pass plans need no scratch) and replayed
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        separate(torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    sep_graph = lat(g.replay, reps)
    del g
    pb.close()
    # the copy bound at the batch's size: one copy of as many bytes (the
    # batch's 2.6 GB each way do not fit the last-level cache, unlike the
    # default workload's 256 MiB)
    cx = torch.empty(total, dtype=torch.uint8, device="cuda")
    cy = torch.empty_like(cx)
    copy_ms, copy_how = best_device_copy(cx, cy, total, stream)
    del cx, cy
    med = float(np.median(resident))

    def p(v, q):
        return round(float(np.percentile(v, q)), 4)
    return {
        "arrays": count, "bytes_per_side": total,
        "GBps": round(gbps(total, med), 1),
        "device_copy_same_bytes_GBps": round(gbps(total, copy_ms), 1),
        "pct_of_device_copy_same_bytes": round(100.0 * copy_ms / med, 1),
        "p50_ms": round(med, 4), "p99_ms": p(resident, 99),
        "oneshot_p50_ms": p(oneshot, 50),
        "oneshot_GBps": round(gbps(total, float(np.median(oneshot))), 1),
        "separate_launches_GBps": round(gbps(total, float(np.median(sep))), 1),
        "separate_p50_ms": p(sep, 50), "separate_p99_ms": p(sep, 99),
        "separate_graph_GBps": round(gbps(total, float(np.median(sep_graph))), 1),
        "separate_graph_p50_ms": p(sep_graph, 50), "separate_graph_p99_ms": p(sep_graph, 99),
        "speedup_vs_separate": round(float(np.median(sep)) / med, 2),
        "speedup_vs_separate_graph": round(float(np.median(sep_graph)) / med, 2),
        "tuned": tuned,
    }


def _bmmc_chunk(specs):
    from synth import gen
    return [gen.random_bmmc(n, sd) for n, sd in specs]


def random_matrices(specs):
    """gen.random_bmmc(n, seed) for every (n, seed), on a few worker
    processes when there are many (started fresh: they never touch the
    GPU)."""
    if len(specs) < 50000:
        return _bmmc_chunk(specs)
    import concurrent.futures as cf
    import multiprocessing as mp
    step = 20000
    chunks = [specs[i:i + step] for i in range(0, len(specs), step)]
    with cf.ProcessPoolExecutor(max_workers=8, mp_context=mp.get_context("spawn")) as ex:
        out = []
        for part in ex.map(_bmmc_chunk, chunks):
            out.extend(part)
    return out


def served_stats(st, reqs, seconds):
    offered = sum((1 << r["n"]) * r["w"] for r in reqs)
    return {"completed": st["completed"], "rejected": st["rejected"],
            "GBps": round(st["bytes_moved"] / max(st["busy_s"], 1e-9) / 1e9, 1),
            "offered_GBps": round(2.0 * offered / reqs[-1]["arrival"] / 1e9, 1),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3), "max_ms": round(st["max_ms"], 3),
            "mean_batch": round(st["mean_batch"], 2), "launches": st["batches"],
            "mean_plan_ms": round(st["mean_plan_ms"], 3), "mean_wait_ms": round(st["mean_wait_ms"], 3),
            "mean_run_ms": round(st["mean_run_ms"], 3), "busy_s": round(st["busy_s"], 3)}


def bench_served(rate=20000.0, seconds=10.0, warm_s=1.0, budget=64 << 30, seed=0, use_graph=0, direct_max=0,
                 solo_log2=0, streams=4, baselines=(1, 4)):
    """Open-loop Poisson arrivals at `rate` requests/s for `seconds` after
    `warm_s` of warm-up requests (other matrices, outside the statistics): n
    uniform in [12, 26], 4- or 8-byte elements, a random BMMC each; inputs
    resident in a pool per (n, width).  The server (continuous batching,
    outputs and scratch from its HBM budget) and then, on the same requests,
    the unbatched baseline: each request its own bmmc_permute at its arrival,
    on 1 and on 4 streams (bmmc_serve_direct; outputs in a buffer per stream
    and size)."""
    import torch
    from paper_2306_07795_amd import binding as B
    from synth import gen
    count = int(rate * seconds)
    reqs = gen.poisson_requests(count, rate, seed, 12, 26, (4, 8))
    warm = gen.poisson_requests(max(1, int(rate * warm_s)), rate, seed + 7919, 12, 26, (4, 8))
    mats = random_matrices([(r["n"], r["seed"]) for r in reqs])
    warm_mats = random_matrices([(r["n"], r["seed"] + 7919) for r in warm])
    pool = {}
    for n in range(12, 27):
        for w in (4, 8):
            pool[(n, w)] = torch.randint(0, 255, ((1 << n) * w,), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def marshal(rs, ms, outs=None, lanes=1):
        return B.DescBatch([(pool[(r["n"], r["w"])], None if outs is None else outs[k % lanes][(r["n"], r["w"])],
                             r["n"], r["w"], m[0], m[1]) for k, (r, m) in enumerate(zip(rs, ms))])

    out = {"rate_req_s": rate, "requests": count, "seconds": seconds, "warmup_s": warm_s}
    srv = B.bmmc_server_create(budget, streams=streams, own_outputs=2, use_graph=use_graph, direct_max=direct_max,
                               solo_log2=solo_log2)
    try:
        # warm-up, then the statistics start afresh; every request is
        # marshalled before the clock starts and submitted ahead of its
        # arrival time (the server plans and launches it only once that time
        # has come), so that the submitting loop never lags behind
        wd = marshal(warm, warm_mats)
        start = B.bmmc_server_now_ns() + int(0.2e9)
        B.bmmc_server_submit_many(srv, wd, [start + int(r["arrival"] * 1e9) for r in warm])
        B.bmmc_server_drain(srv)
        B.bmmc_server_reset_stats(srv)
        descs = marshal(reqs, mats)
        lead = max(5.0, 1.0 + 1.2e-5 * count)  # submitting takes about 7-9 us per request
        start = B.bmmc_server_now_ns() + int(lead * 1e9)
        B.bmmc_server_submit_many(srv, descs, [start + int(r["arrival"] * 1e9) for r in reqs])
        submit_s = (B.bmmc_server_now_ns() - start) * 1e-9 + lead
        if submit_s >= lead:
            raise SystemExit(f"bench: submitting took {submit_s:.2f} s, beyond the {lead} s lead")
        B.bmmc_server_drain(srv)
        st = B.bmmc_server_stats(srv)
    finally:
        B.bmmc_server_destroy(srv)
    out.update(served_stats(st, reqs, seconds))
    out["peak_budget_GB"] = round(st["peak_bytes"] / 1e9, 2)
    out["streams"] = streams
    del descs
    torch.cuda.empty_cache()
    for lanes in baselines:
        outs = [{(n, w): torch.empty((1 << n) * w, dtype=torch.uint8, device="cuda")
                 for n in range(12, 27) for w in (4, 8)} for _ in range(lanes)]
        wd = marshal(warm, warm_mats, outs, lanes)
        start = B.bmmc_server_now_ns() + int(0.2e9)
        B.bmmc_serve_direct(wd, [start + int(r["arrival"] * 1e9) for r in warm], lanes)
        d = marshal(reqs, mats, outs, lanes)
        start = B.bmmc_server_now_ns() + int(0.2e9)
        st = B.bmmc_serve_direct(d, [start + int(r["arrival"] * 1e9) for r in reqs], lanes)
        out[f"per_request_{lanes}_stream{'s' if lanes > 1 else ''}"] = served_stats(st, reqs, seconds)
        del outs, d, wd
        torch.cuda.empty_cache()
    return out


def transpose_sweep(n=25, w=4, steps=10):
    """The paper's AMD experiment (Section 6, transpose time against the
    number of columns at a fixed 2^25 elements), on this GPU: for every split
    k, the 2^(n-k) x 2^k matrix transpose (bit-block swap, one tiled pass) by
    the library's default call, the naive kernel and the device copy, each
    call after a cache flush (as the headline); the tiled pass's own kernel
    duration from events bound to its launches."""
    import torch
    from paper_2306_07795_amd import binding as B
    from synth import gen
    nbytes = (1 << n) * w
    x = torch.from_numpy(gen.data(n, w, 0).view("uint8")).to("cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    flush = Flusher(x.device)
    copy_ms, copy_how = best_device_copy(x, y, nbytes, stream, flush)
    table = []
    for k in range(n + 1):
        rows = gen.block_swap_rows(n, k)
        call = lambda: B.bmmc_permute(x, y, n, rows, 0, w, stream)  # noqa: E731
        t_ms = mean(flushed_times(call, steps, 2, stream, flush))
        kname, ks = profiled_kernels(call, steps, stream, flush)
        nv_ms = mean(flushed_times(lambda: B.bmmc_permute_naive(x, y, n, rows, 0, w, stream), 3, 1, stream, flush))
        table.append({"k": k, "columns": 1 << k, "rows": 1 << (n - k),
                      "tiled_us": round(t_ms * 1e3, 2), "tiled_GBps": round(gbps(nbytes, t_ms), 1),
                      "tiled_pct_of_copy": round(100.0 * copy_ms / t_ms, 1),
                      "kernel": kname, "kernel_us": round(1e3 * ks["total_ms"] / ks["launches"], 2),
                      "naive_us": round(nv_ms * 1e3, 2), "naive_GBps": round(gbps(nbytes, nv_ms), 1)})
        progress(f"transpose k={k}: {table[-1]['tiled_pct_of_copy']} % of copy")
    return {"n": n, "elem_bytes": w, "cache_state": "flushed before every call", "copy_us": round(copy_ms * 1e3, 2),
            "copy": copy_how, "table": table}


def sortnet_table(sizes=(12, 16, 20, 24, 26), seed=0):
    """The sorting network of Section 7.1 on 2^n int32 keys: compiled to
    coalesced BMMC passes with the compare-exchange fused into each pass, and
    run directly at the keys' positions; torch.sort beside them for context
    (and as the sanity check before timing; parity is the tests' job)."""
    import numpy as np
    import torch
    from paper_2306_07795_amd import binding as B
    stream = torch.cuda.current_stream()
    rows = []
    for n in sizes:
        rng = np.random.default_rng(seed + n)
        a = rng.integers(-(1 << 31), 1 << 31, size=1 << n, dtype=np.int64).astype(np.int32)
        x = torch.from_numpy(a).to("cuda")
        y = torch.empty_like(x)
        want = torch.sort(x).values
        npass, most = B.bmmc_sortnet_passes(n)
        ent = {"n": n, "keys": 1 << n, "columns": n * (n + 1) // 2, "passes": npass,
               "most_columns_per_pass": most}
        for name, m in (("passes", B.SORTNET_PASSES), ("direct", B.SORTNET_DIRECT)):
            B.bmmc_sortnet(x, y, n, B.KEY_I32, m, stream)
            torch.cuda.synchronize()
            if not torch.equal(y, want):
                raise SystemExit(f"sortnet {name} n={n}: output differs from torch.sort")
            reps = 20 if n <= 20 else 5
            ms = timed(lambda: B.bmmc_sortnet(x, y, n, B.KEY_I32, m, stream), reps, 1, stream)
            # every pass (direct: every column, plus the first copy) reads and
            # writes the whole array once
            launches = npass if m == B.SORTNET_PASSES else ent["columns"] + 1
            ent[f"{name}_ms"] = round(ms, 4)
            ent[f"{name}_launch_GBps"] = round(2.0 * launches * a.nbytes / (ms * 1e-3) / 1e9, 1)
        ms = timed(lambda: torch.sort(x), 20 if n <= 20 else 5, 1, stream)
        ent["torch_sort_ms"] = round(ms, 4)
        ent["passes_speedup_vs_direct"] = round(ent["direct_ms"] / ent["passes_ms"], 2)
        rows.append(ent)
        del x, y
    return {"workload": "sorting network (even/odd merge, balanced periodic merger) on int32 keys",
            "table": rows}


CACHE_RESIDENT_BYTES = 64 << 20


def sanity(B, x, y, n, rows, c, w, step, stream):
    """What is timed is a permutation of the input: the inverse, run by the
    library's default path, restores it (parity with the oracle is the
    tests' job)."""
    import torch
    step()
    inv_rows, inv_c = B.bmmc_invert(rows, c, n)
    z = torch.empty_like(x)
    B.bmmc_permute(y, z, n, inv_rows, inv_c, w, stream)
    torch.cuda.synchronize()
    if not torch.equal(z, x):
        print("bench: the inverse permutation does not restore the input", file=sys.stderr)
        sys.exit(1)
    del z


def graph_time(fn, steps, warmup):
    """Mean time of fn() when `steps` calls are captured once into a HIP graph
    (torch's capture; the calls enqueue on the capture stream) and the timed
    region is one replay of it."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(warmup):
            fn(side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = torch.cuda.current_stream()
        for _ in range(steps):
            fn(cap)
    g.replay()  # warm replay
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    g.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def graph_timed_line(args, n, w, rows, c, opts, tuned, desc, x, y, nbytes, passes, stream):
    """Arrays that stay in the caches run for a few microseconds, less than
    what one host call costs: the steps, and the copy they are compared with,
    are timed as one replay of a graph of the calls.  The per-launch duration
    is the replay time divided by the launches in it."""
    from paper_2306_07795_amd import binding as B
    ms = graph_time(lambda s: B.bmmc_permute_ex(x, y, n, rows, c, w, opts, s), args.steps, args.warmup)
    value = gbps(nbytes, ms)
    copy_ms, copy_how = 1e30, None
    for vpt in (1, 2, 4, 8):
        for hints in (0, 1, 2, 3):
            t = graph_time(lambda s: B.bmmc_copy_ex(x, y, nbytes, vpt, hints, s), args.steps, 2)
            copy_ms, copy_how = min((copy_ms, copy_how), (t, f"k_copy vpt={vpt} hints={hints} (graph)"))
    dev_copy = gbps(nbytes, copy_ms)
    per_launch_ms = ms / passes
    achieved = 2.0 * nbytes / (per_launch_ms * 1e-3) / 1e9
    return print(json.dumps({
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "elem_bytes": w, "method": args.method, "passes": passes,
                   "seed": 0, "options": tuned, "timing": "one replay of a graph of the steps (cache resident)"},
        "pct_of_device_copy": round(100.0 * value / dev_copy, 2),
        "pct_of_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "device_copy_GBps": round(dev_copy, 1), "device_copy": copy_how,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                     "kernel": "tiled pass (graph replay; per-launch time = replay / launches)",
                     "mean_launch_ms": round(per_launch_ms, 5), "bytes_per_launch": 2.0 * nbytes},
    }), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="random26", choices=sorted(WORKLOADS))
    ap.add_argument("--method", default="auto", choices=["auto", "tiled", "onepass", "naive"])
    ap.add_argument("--seed", type=int, default=0, help="seed of the random matrix (random workloads)")
    ap.add_argument("--no-tune", action="store_true", help="time the library defaults, no autotuning")
    ap.add_argument("--retune", action="store_true",
                    help="autotune now instead of taking the options from the tuning file")
    ap.add_argument("--save-tune", metavar="PATH",
                    help="merge this run's tuning into the JSON-lines file PATH")
    ap.add_argument("--options-from", metavar="BENCH_JSON",
                    help="no autotuning: take the options from the JSON line of an earlier run")
    ap.add_argument("--default-call", action="store_true",
                    help="time the call without options (bmmc_permute's own choice) instead of the tuning "
                         "file's options for the matrix's class")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed permutation and the copy bound (for counter runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-rate", type=float, default=20000.0)
    ap.add_argument("--served-seconds", type=float, default=10.0)
    ap.add_argument("--extras-out", default=None, help="write extra measurements (JSON) here")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc runs of this "
                         "benchmark (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--transpose-sweep", action="store_true",
                    help="print the transpose-vs-columns table at 2^25 int32 and exit")
    ap.add_argument("--sortnet", action="store_true",
                    help="print the sorting-network table (compiled passes vs direct) and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="print the batched form's measurement (1024 arrays) and exit")
    ap.add_argument("--served-sweep", action="store_true",
                    help="print the served form and its per-request baselines at 10k-80k requests/s and exit")
    args = ap.parse_args()
    if args.transpose_sweep:
        print(json.dumps(transpose_sweep()), flush=True)
        return
    if args.sortnet:
        print(json.dumps(sortnet_table()), flush=True)
        return
    if args.batched_only:
        print(json.dumps(bench_batched(retune=args.retune)), flush=True)
        return
    if args.served_sweep:
        rows = []
        for rate in (10000.0, 20000.0, 40000.0, 60000.0, 80000.0):
            rows.append(bench_served(rate, args.served_seconds))
            progress(f"served at {rate:.0f} requests/s: {json.dumps(rows[-1])}")
        print(json.dumps({"workload": "served load sweep: server (4 streams) against per-request launches on "
                                      "1 and 4 streams, same Poisson requests", "table": rows}), flush=True)
        return
    # entry of profiles/traffic.json: the workload, and the method unless it is the default
    traffic_key = args.workload + ("" if args.method == "auto" else "_" + args.method)
    if args.traffic_from:
        n, w = WORKLOADS[args.workload][:2]
        print(json.dumps(write_traffic(args.traffic_from[0], args.traffic_from[1], (1 << n) * w, traffic_key),
                         indent=1))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2306_07795_amd import binding as B
    from synth import gen

    n, w, kind, desc = WORKLOADS[args.workload]
    rows, c = matrix(kind, n, args.seed)
    method = {"auto": B.METHOD_AUTO, "tiled": B.METHOD_TILED, "onepass": B.METHOD_ONEPASS,
              "naive": B.METHOD_NAIVE}[args.method]

    a = gen.data(n, w, 0)
    nbytes = a.nbytes
    dev = torch.device("cuda:0")
    x = torch.from_numpy(a.view(np.uint8).reshape(-1)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()

    if args.save_tune and os.path.exists(args.save_tune):
        B.bmmc_tune_load(args.save_tune)
    elif not (args.retune or args.no_tune) and os.path.exists(TUNE_DB):
        B.bmmc_tune_load(TUNE_DB)
    opts = {"method": method}
    tuned, tuning = None, "library defaults"
    if args.options_from:
        with open(args.options_from) as fh:
            tuned = json.loads(fh.read().strip().splitlines()[-1])["config"]["options"]
        tuning = "options of an earlier run"
    elif not args.no_tune and method != B.METHOD_NAIVE:
        # the tuned options of this matrix's class (tiled or not)
        tuned, tuning = (None if args.retune else B.bmmc_tune_lookup(n, w, rows, method)), "tuning file"
        if tuned is None:
            B.bmmc_autotune(n, w, method, stream, 3)
            tuned, tuning = B.bmmc_tune_lookup(n, w, rows, method), "autotuned in this run"
    if tuned:
        opts = dict(tuned)
    if args.default_call:
        # no options: what bmmc_permute does by itself (its class's tuned
        # options, and above 256 MiB dealt output blocks for matrices that
        # keep their 4 KiB-block bits)
        opts, tuned, tuning = None, None, "none given: the library's default call"
    passes = B.bmmc_plan_ex(rows, c, n, w, opts).nfactors

    def step():
        B.bmmc_permute_ex(x, y, n, rows, c, w, opts, stream)

    if nbytes < CACHE_RESIDENT_BYTES:
        sanity(B, x, y, n, rows, c, w, step, stream)
        graph_timed_line(args, n, w, rows, c, opts, tuned, desc, x, y, nbytes, passes, stream)
        if args.save_tune:
            B.bmmc_tune_save(args.save_tune)
        return

    # timed region: exactly `steps` permutations, each right after a cache
    # flush (outside the timed interval); HIP events on the stream around
    # each step.  Then the same steps again with the library's profiling on:
    # it binds a second pair of events to every kernel it launches, which
    # gives each launch's own duration (the roofline), but its bookkeeping
    # would lengthen the steps, so it stays out of the timed steps.
    flush = Flusher(dev)
    for _ in range(args.warmup):
        flush(stream)
        step()
    torch.cuda.synchronize()
    evs = []
    for _ in range(args.steps):
        flush(stream)
        ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea.record(stream)
        step()
        eb.record(stream)
        evs.append((ea, eb))
    torch.cuda.synchronize()
    B.bmmc_profile_begin()
    for _ in range(args.steps):
        flush(stream)
        step()
    torch.cuda.synchronize()
    kstats = B.bmmc_profile_end()
    step_ms = [ea.elapsed_time(eb) for ea, eb in evs]
    ms = mean(step_ms)
    value = gbps(nbytes, ms)
    progress(f"timed steps: {ms:.5f} ms per step, {value:.1f} GB/s (flushed)")

    # the copy bound in the same state and session
    copy_ms, copy_how = best_device_copy(x, y, nbytes, stream, flush)
    dev_copy = gbps(nbytes, copy_ms)
    extras = {"device_copy": copy_how, "step_ms_min": round(min(step_ms), 5),
              "step_ms_max": round(max(step_ms), 5)}
    if not args.no_extras:
        # the steady state of one call repeated on the same buffers (part of
        # an array that fits the 256 MB last-level cache stays there between
        # calls), against a copy repeated the same way
        warm_ms = timed(step, args.steps, args.warmup, stream)
        B.bmmc_profile_begin()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        wname, wk = dominant(B.bmmc_profile_end())
        warm_copy_ms, warm_copy_how = best_device_copy(x, y, nbytes, stream)
        extras["warm"] = {"GBps": round(gbps(nbytes, warm_ms), 1), "ms_per_step": round(warm_ms, 5),
                          "device_copy_GBps": round(gbps(nbytes, warm_copy_ms), 1), "device_copy": warm_copy_how,
                          "pct_of_device_copy": round(100.0 * warm_copy_ms / warm_ms, 2),
                          "kernel": wname, "kernel_mean_launch_ms": round(wk["total_ms"] / wk["launches"], 5)}
    # the traffic calibration kernel, k_copy<4,0>, launched at least once
    B.bmmc_copy_ex(x, y, nbytes, 4, 0, stream)
    if method == B.METHOD_AUTO and not args.no_extras:
        naive_ms = mean(flushed_times(lambda: B.bmmc_permute_naive(x, y, n, rows, c, w, stream), 5, 1, stream,
                                      flush))
        extras["naive_GBps"] = round(gbps(nbytes, naive_ms), 1)
        extras["paper_two_pass"] = paper_two_pass(x, y, n, rows, c, w, stream, flush, copy_ms, warm_copy_ms,
                                                  tune=not (args.no_tune or args.options_from),
                                                  retune=args.retune)
        extras["cache_state"] = cache_states(x, y, n, rows, c, w, opts, extras["paper_two_pass"]["options"],
                                             stream, flush)
        if kind == "random":
            extras["random_matrices"] = other_matrices(x, y, n, w, copy_ms, stream, flush)
    # parity with the oracle is the tests' job; this checks that what was
    # timed is a permutation of the input: the inverse, by the library's
    # default path, restores it
    sanity(B, x, y, n, rows, c, w, step, stream)

    # roofline of the dominant kernel: algorithmic bytes per launch / its
    # mean launch duration (kernel-bound events of the timed steps)
    dname, d = dominant(kstats)
    per_launch_ms = d["total_ms"] / d["launches"]
    launch_bytes = d["bytes"] / d["launches"]
    achieved = launch_bytes / (per_launch_ms * 1e-3) / 1e9
    tbytes = traffic_for(traffic_key, dname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4),
                # HBM bytes per launch from the rocprofv3 counters, as a rate over the same launch time
                "traffic": None if tbytes is None else round(tbytes / (per_launch_ms * 1e-3) / 1e9, 1),
                "traffic_bytes_per_launch": tbytes,
                "kernel": dname, "launches": d["launches"], "mean_launch_ms": round(per_launch_ms, 5),
                "launch_time_from": "events bound to each launch (hipExtLaunchKernel) of a second, profiled "
                                    "run of the timed steps",
                "cache_state": "flushed before every step",
                "bytes_per_launch": launch_bytes}

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "elem_bytes": w, "method": args.method,
                   "passes": passes, "seed": args.seed, "options": tuned, "tuning": tuning,
                   "cache_state": f"flushed: a {FLUSH_BYTES >> 20} MiB copy between two other buffers before "
                                  "every step, outside the timed interval (the copy bound likewise)"},
        "pct_of_device_copy": round(100.0 * value / dev_copy, 2),
        "pct_of_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "device_copy_GBps": round(dev_copy, 1),
        "traffic_GBps": round(value * passes, 2),
        "traffic_pct_of_device_copy": round(100.0 * value * passes / dev_copy, 2),
        "roofline": roofline,
        "extras": extras,
    }
    del x, y, flush
    torch.cuda.empty_cache()
    progress("single-array extras done")
    if not args.no_batched and not args.no_extras:
        line["batched"] = bench_batched(retune=args.retune)
        torch.cuda.empty_cache()
        progress("batched done")
    if not args.no_served and not args.no_extras:
        line["served"] = bench_served(args.served_rate, args.served_seconds)
        torch.cuda.empty_cache()
        progress("served done")
        # past the capacity: the same mix at 60k requests/s for 5 s, where
        # continuous batching carries more than per-request launches
        line["served_overload"] = bench_served(3.0 * args.served_rate, args.served_seconds / 2, baselines=(4,))
        torch.cuda.empty_cache()
        progress("served past capacity done")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(a, n, rows, c)
    if args.extras_out:
        with open(args.extras_out, "w") as f:
            json.dump({"kernels": kstats, **extras}, f, indent=1)
    if args.save_tune:
        B.bmmc_tune_save(args.save_tune)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
