#!/usr/bin/env python3
"""Throughput of BMMC permutations on one MI355X.

Default workload: a uniformly random invertible 26 x 26 matrix over F_2 with
a random complement (seed 0), applied to 2^26 int32 elements drawn from seed
0 -- the paper's scheme, i.e. two LDS-staged tiled passes through scratch.
One step is one whole permutation (both passes) of the resident array.

Prints ONE JSON line.  `value` is effective throughput in GB/s (decimal):
algorithmic bytes (one read + one write of the array, 2 * 2^n * w) per step
time.  Beside it: the same-session device-copy rate and HBM peak fractions,
the traffic rate (bytes of both passes), the per-kernel roofline of the tiled
pass, and the CPU oracle's rate on this host.
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
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    # name: (n, elem_bytes, matrix kind, description)
    "random26": (26, 4, "random", "random BMMC on 2^26 int32 (A uniform invertible 26x26 over F_2, random c, seed 0)"),
    "random28": (28, 4, "random", "random BMMC on 2^28 int32 (seed 0)"),
    "random27x8": (27, 8, "random", "random BMMC on 2^27 int64 (seed 0)"),
    "bitrev28": (28, 4, "bitrev", "bit reversal of 2^28 int32"),
    "swap28": (28, 4, "swap", "2^14 x 2^14 int32 matrix transpose (low/high bit-block swap)"),
    "bitrev20": (20, 4, "bitrev", "bit reversal of 2^20 int32 (cache resident)"),
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


def cpu_baseline(a, n, rows, c, w, budget_s=12.0):
    """The oracle, as is, on this host's cores: repeats of the full workload
    until about budget_s seconds have passed (at least one)."""
    from oracle import oracle as orc
    cores = orc.threads(0)
    reps, t0 = 0, time.perf_counter()
    while True:
        orc.permute(a, n, rows, c, 0)
        reps += 1
        if time.perf_counter() - t0 > budget_s or reps >= 20:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": round(2.0 * a.nbytes / dt / 1e9, 3), "unit": "GB/s", "cores": cores,
            "kind": "oracle",
            "sample": f"the full workload (2^{n} elements), {reps} repetition(s), {dt:.2f} s each"}


def traffic_for(kernel, launch_bytes):
    """HBM bytes per launch measured with rocprofv3 counters, if they were taken
    on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel)
    if not ent:
        return None
    return ent.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="random26", choices=sorted(WORKLOADS))
    ap.add_argument("--method", default="auto", choices=["auto", "onepass", "naive"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--extras-out", default=None, help="write extra measurements (JSON) here")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2306_07795_amd import binding as B
    from synth import gen

    n, w, kind, desc = WORKLOADS[args.workload]
    rows, c = matrix(kind, n)
    method = {"auto": B.METHOD_AUTO, "onepass": B.METHOD_ONEPASS, "naive": B.METHOD_NAIVE}[args.method]
    plan = B.bmmc_factorize_t(rows, c, n, 0, w) if method == B.METHOD_AUTO else None
    passes = plan.nfactors if plan is not None else 1

    a = gen.data(n, w, 0)
    nbytes = a.nbytes
    dev = torch.device("cuda:0")
    x = torch.from_numpy(a.view(np.uint8).reshape(-1)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    opts = {"method": method}

    def step():
        B.bmmc_permute_ex(x, y, n, rows, c, w, opts, stream)

    # correctness of what is timed: sampled outputs against the oracle
    step()
    torch.cuda.synchronize()
    from oracle import oracle as orc
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 1 << n, size=4096, dtype=np.uint64)
    ys = orc.apply_many(rows, c, n, xs).astype(np.int64)
    got = y.cpu().numpy().view(a.dtype).reshape(a.shape)
    if not np.array_equal(got[ys], a[xs.astype(np.int64)]):
        print("bench: output differs from the oracle", file=sys.stderr)
        sys.exit(1)

    # timed region: exactly `steps` permutations, per-launch events on the stream
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    B.bmmc_profile_begin()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    kstats = B.bmmc_profile_end()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = 2.0 * nbytes / (ms * 1e-3) / 1e9

    # bounds in the same session: copy kernel, hipMemcpy D2D, naive kernel
    copy_ms = timed(lambda: B.bmmc_copy(x, y, nbytes, stream), 20, 3, stream)
    d2d_ms = timed(lambda: y.copy_(x), 20, 3, stream)
    dev_copy_gbps = 2.0 * nbytes / (min(copy_ms, d2d_ms) * 1e-3) / 1e9
    extras = {
        "copy_kernel_GBps": round(2.0 * nbytes / (copy_ms * 1e-3) / 1e9, 1),
        "hipmemcpy_d2d_GBps": round(2.0 * nbytes / (d2d_ms * 1e-3) / 1e9, 1),
    }
    if method == B.METHOD_AUTO:
        naive_ms = timed(lambda: B.bmmc_permute_naive(x, y, n, rows, c, w, stream), 10, 2, stream)
        one_ms = timed(lambda: B.bmmc_permute_ex(x, y, n, rows, c, w, {"method": B.METHOD_ONEPASS},
                                                 stream), 20, 3, stream)
        extras["naive_GBps"] = round(2.0 * nbytes / (naive_ms * 1e-3) / 1e9, 1)
        extras["onepass_GBps"] = round(2.0 * nbytes / (one_ms * 1e-3) / 1e9, 1)
        extras["onepass_pct_of_device_copy"] = round(100.0 * extras["onepass_GBps"] / dev_copy_gbps, 2)

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    dom = max(kstats.items(), key=lambda kv: kv[1]["total_ms"])
    dname, d = dom
    per_launch_ms = d["total_ms"] / d["launches"]
    launch_bytes = d["bytes"] / d["launches"]
    achieved = launch_bytes / (per_launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic_for(dname, launch_bytes),
                "kernel": dname, "launches": d["launches"], "mean_launch_ms": round(per_launch_ms, 5),
                "bytes_per_launch": launch_bytes}

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "elem_bytes": w, "method": args.method,
                   "passes": passes, "seed": 0},
        "pct_of_device_copy": round(100.0 * value / dev_copy_gbps, 2),
        "pct_of_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "device_copy_GBps": round(dev_copy_gbps, 1),
        "traffic_GBps": round(value * passes, 2),
        "traffic_pct_of_device_copy": round(100.0 * value * passes / dev_copy_gbps, 2),
        "roofline": roofline,
        "extras": extras,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(a, n, rows, c, w)
    if args.extras_out:
        with open(args.extras_out, "w") as f:
            json.dump({"kernels": kstats, **extras}, f, indent=1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
