"""Pick a setting for a class of matrices by its worst case over many of them.

Beyond the last-level cache the rate of one setting differs from one random
matrix to the next, and a setting chosen on a few matrices can leave some
matrix far behind.  This script times a grid of settings (tile shape, read
and write runs, tile order; non-temporal loads, cached stores) on the random
matrices of several seeds, each call after a 512 MiB cache flush, and writes
the setting with the best worst case (ties: the best mean) as the entry of
this size for random matrices and the default method in a tuning file.
With --matrices bpc it does the same for the class of tiled matrices, on bit
permutations: the bit reversal, the transposes of 2^(n/2) x 2^(n-n/2) and
2^7 x 2^(n-7) elements and the random bit permutations of the seeds.  The
shipped file's tiled-class entries are the autotuner's, not this mode's:
its pick raises the worst random bit permutation but lowers the bit
reversal and the transposes by 6-8 points of the copy at 1 GiB.

    python paper_2306_07795_amd/tuning/sweep_robust.py --n 28 --w 4 --seeds 0-7,100-107 \
        --out paper_2306_07795_amd/tuning/gfx950.jsonl
    python paper_2306_07795_amd/tuning/sweep_robust.py --n 28 --w 4 --matrices bpc --seeds 0-3 \
        --out paper_2306_07795_amd/tuning/gfx950.jsonl

Every timed call's result is compared by the tests, not here.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

FLUSH_BYTES = 512 << 20


def seeds_of(spec):
    out = []
    for part in spec.split(","):
        lo, _, hi = part.partition("-")
        out.extend(range(int(lo), int(hi or lo) + 1))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--w", type=int, required=True)
    ap.add_argument("--seeds", default="0-7,100-107")
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--matrices", choices=("random", "bpc"), default="random")
    ap.add_argument("--out", required=True, help="tuning file whose entry is replaced")
    args = ap.parse_args()

    import numpy as np
    import torch
    from paper_2306_07795_amd import binding as B
    from synth import gen

    n, w = args.n, args.w
    stream = torch.cuda.current_stream()
    fa = torch.full((FLUSH_BYTES,), 0x3C, dtype=torch.uint8, device="cuda")
    fb = torch.empty_like(fa)
    a = gen.data(n, w, 0)
    x = torch.from_numpy(a.view(np.uint8).reshape(-1)).to("cuda")
    y = torch.empty_like(x)

    def flushed_ms(fn):
        ts = []
        for r in range(args.reps + 1):
            B.bmmc_copy_ex(fa, fb, FLUSH_BYTES, 1, 0, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            ts.append((e0, e1))
        torch.cuda.synchronize()
        v = [e0.elapsed_time(e1) for e0, e1 in ts[1:]]
        return sum(v) / len(v)

    copy_ms = min(flushed_ms(lambda vpt=vpt: B.bmmc_copy_ex(x, y, a.nbytes, vpt, 1, stream)) for vpt in (1, 2, 4))
    if args.matrices == "random":
        cls = 0
        mats = [gen.random_bmmc(n, s) for s in seeds_of(args.seeds)]
        orders = (4, 4 + 16 * 7, 3, 1, 1 + 16 * 12, 2)
        shapes = [(512, 2), (256, 4), (512, 4), (256, 8), (1024, 4), (512, 8)]
    else:
        cls = 1
        mats = [(gen.bit_reversal_rows(n), 0), (gen.block_swap_rows(n, n // 2), 0), (gen.block_swap_rows(n, 7), 0)]
        mats += [gen.random_bpc(n, s) for s in seeds_of(args.seeds)]
        orders = (4, 4 + 16 * 7, 1, 1 + 16 * 7, 2, 3)
        shapes = [(512, 2), (256, 4), (512, 4), (256, 8), (1024, 4), (512, 8), (256, 16)]
    lv = {4: 2, 8: 1}[w]
    min_run = {4: 5, 8: 4}[w]  # runs of at least one 128-byte line
    best = None
    for nt, it in shapes:
        D = lv + nt.bit_length() - 1 + it.bit_length() - 1
        for ra in range(min_run, D - min_run + 1):
            rb = D - ra
            for order in orders:
                o = {"method": 0, "threads": nt, "iters": it, "t": min(ra, rb), "run_in": ra, "run_out": rb,
                     "hints": 1, "swizzle": 1, "tile_order": order, "grid": -1}
                try:
                    pcts = [100.0 * copy_ms / flushed_ms(lambda r=r, c=c: B.bmmc_permute_ex(x, y, n, r, c, w, o,
                                                                                           stream))
                            for r, c in mats]
                except B.BmmcError:
                    continue  # no kernel of this shape, or the runs do not fit
                score = (min(pcts), sum(pcts) / len(pcts))
                print(json.dumps({"options": o, "min": round(score[0], 1), "mean": round(score[1], 1),
                                  "pcts": [round(v, 1) for v in pcts]}), flush=True)
                if best is None or score > best[0]:
                    best = (score, o)
    (worst, mean), o = best
    ms = copy_ms * 100.0 / mean  # the mean time per call
    lines = open(args.out).read().splitlines()
    out = []
    for line in lines:
        d = json.loads(line)
        if (d.get("kind") == "plain" and d["n"] == n and d["w"] == w and d["method"] == 0 and d["class"] == cls):
            d.update({k: o[k] for k in ("threads", "iters", "t", "run_in", "run_out", "hints", "tile_order", "grid",
                                         "swizzle")})
            d["ms"] = round(ms, 6)
            line = json.dumps(d)
        out.append(line)
    with open(args.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(f"n={n} w={w} {args.matrices}: worst {worst:.1f} %, mean {mean:.1f} % of the flushed copy over "
          f"{len(mats)} matrices: {o}", flush=True)


if __name__ == "__main__":
    main()
