"""Regenerate a tuning file with the library's own autotuner.

Runs bmmc_autotune for every array size of 4- and 8-byte elements from one
tile to 1 GiB, for the default method (random matrices and bit permutations,
stored as two classes) and for the two-pass scheme of Section 5.2 at the
larger sizes, then writes the tuning cache as JSON lines.  The library loads
`gfx950.jsonl` beside this script on first use.  With --batched, it instead
tunes the batched kernel for the benchmark's batch (1024 arrays of 2^10-2^22
int32 elements) and merges that entry into the file PATH.

    BMMC_TUNE_CACHE= python paper_2306_07795_amd/tuning/make_tuning.py --out PATH
    python paper_2306_07795_amd/tuning/make_tuning.py --batched --out PATH

With BMMC_TUNE_CACHE=PATH the library also writes PATH after every size it
tunes; with BMMC_TUNE_VERBOSE=1 it reports every 32 timed settings on stderr
(a 1 GiB size takes minutes).  The shipped file's entries for random
matrices of 1 GiB (n = 28 int32, n = 27 int64) then come from
`sweep_robust.py` beside this script, which picks by the worst case over
sixteen matrices.
"""
import argparse
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from paper_2306_07795_amd import binding as B  # noqa: E402


def tune_batched(reps):
    """The benchmark's batch: 1024 int32 arrays, n uniform in [10, 22] (the
    entry is keyed by the histogram of sizes, so the data and matrices only
    have to be valid)."""
    import torch
    from synth import gen
    sizes = gen.batched_sizes(1024, 0, 10, 22)
    items = []
    for k, n in enumerate(sizes):
        rows, c = gen.random_bmmc(n, 1_000_003 + k)
        x = torch.zeros(1 << n, dtype=torch.int32, device="cuda")
        items.append((x, torch.empty_like(x), n, 4, rows, c))
    t0 = time.time()
    opts, ms = B.bmmc_autotune_batched(items, torch.cuda.current_stream(), reps)
    total = sum((1 << n) * 4 for n in sizes)
    print(f"batched 1024 arrays: {ms:.4f} ms ({2.0 * total / (ms * 1e-3) / 1e9:.0f} GB/s) "
          f"in {time.time() - t0:.1f} s  {opts}", flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True, help="tuning file to write (JSON lines)")
    ap.add_argument("--widths", default="4,8", help="element widths in bytes")
    ap.add_argument("--max-bytes-log2", type=int, default=30, help="largest array: 2^this bytes")
    ap.add_argument("--min-n", type=int, default=12, help="smallest n")
    ap.add_argument("--tiled-from-log2", type=int, default=24,
                    help="also tune the two-pass scheme from arrays of 2^this bytes")
    ap.add_argument("--reps", type=int, default=3, help="timed calls per candidate from 64 MiB on")
    ap.add_argument("--reps-small", type=int, default=20,
                    help="timed calls per candidate below 64 MiB (captured into one graph)")
    ap.add_argument("--batched", action="store_true",
                    help="only tune the benchmark's batch and merge it into --out")
    args = ap.parse_args()
    if args.batched:
        if os.path.exists(args.out):
            B.bmmc_tune_load(args.out)
        tune_batched(args.reps)
        B.bmmc_tune_save(args.out)
        print("wrote", args.out, flush=True)
        return
    if os.environ.get("BMMC_TUNE_CACHE", None) != "":
        print("note: BMMC_TUNE_CACHE is not empty; the entries of that file are kept", flush=True)
    for w in (int(v) for v in args.widths.split(",")):
        lw = w.bit_length() - 1
        for n in range(args.min_n, args.max_bytes_log2 - lw + 1):
            methods = [B.METHOD_AUTO]
            if n + lw >= args.tiled_from_log2:
                methods.append(B.METHOD_TILED)
            reps = args.reps if (1 << (n + lw)) >= (64 << 20) else args.reps_small
            for m in methods:
                t0 = time.time()
                opts, ms = B.bmmc_autotune(n, w, m, None, reps)
                gbps = 2.0 * (1 << n) * w / (ms * 1e-3) / 1e9
                print(f"n={n} w={w} method={m}: {ms:.4f} ms ({gbps:.0f} GB/s) in {time.time() - t0:.1f} s  {opts}",
                      flush=True)
    B.bmmc_tune_save(args.out)
    print("wrote", args.out, flush=True)


if __name__ == "__main__":
    main()
