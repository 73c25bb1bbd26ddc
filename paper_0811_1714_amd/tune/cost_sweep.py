"""Timing sweep for the fixed cost model that picks a schedule for large products (at
least 2^30 bit-operations) when no model or autotune result is in use: every M4RM
schedule the default chooses from (tile, Strassen-Winograd cutoff, k split) timed on
squares from 1024 to 32768 and on rectangles, one JSON line per schedule.  The first line
of each shape is the library's own choice.

    python -m paper_0811_1714_amd.tune.cost_sweep --out cost_sweep.jsonl

``fit_cost`` fits the per-tile-family constants of the cost model to the result.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Tiles the default chooses from (library variant numbers).
VARIANTS = (0, 10, 1, 2, 3, 4, 11, 12, 13, 14, 15, 16, 17, 18)
SHAPES = [(1024,) * 3, (2048,) * 3, (3000,) * 3, (4096,) * 3, (6000,) * 3, (8192,) * 3, (12000,) * 3,
          (16384,) * 3, (10000, 20000, 5000), (20001, 777, 30003), (4095, 65537, 129), (12000, 6000, 12000),
          (3000, 50000, 3000), (30000, 2000, 30000), (8192, 8192, 1024), (1024, 8192, 8192), (8192, 1024, 8192),
          (16384, 4096, 16384), (4096, 16384, 4096), (2000, 2000, 60000), (60000, 2000, 2000), (32768,) * 3]


def words(c):
    return (c + 63) // 64


def splittable(m, k, n, cutoff):
    c = max(cutoff, 64)
    return cutoff > 0 and m > c and k > c and n > c


def small_shapes(count=48, seed=11):
    """Products below 2^30 bit-operations drawn from the batched workload's law (m, k, n
    log-uniform in [64, 4096)), plus three fixed squares."""
    import synth
    dims = synth.log_uniform_dims(seed, 77, 4 * count, 64, 4096)
    out = [(512,) * 3, (256,) * 3, (768,) * 3]
    for m, k, n in dims:
        if m * k * n < 2 ** 30 and len(out) < count:
            out.append((int(m), int(k), int(n)))
    return out


HUGE_SHAPES = [(65536,) * 3]


def candidates(m, k, n, min_slice_words=16):
    """(variant, cutoff, k split) triples the default considers for the shape: cutoffs of
    min(m, k, n) / 2, / 4, / 8 of at least 2048, k split only without recursion and with
    at least ``min_slice_words`` words of k per slice."""
    mn = min(m, k, n)
    out = []
    for c in (0, mn // 2, mn // 4, mn // 8):
        if c and (c < 2048 or not splittable(m, k, n, c)):
            continue
        for v in VARIANTS:
            if m * k * n >= 2 ** 45 and c == 0 and v not in (16, 10):
                continue                      # no recursion at 32768^3: two tiles suffice
            if m * k * n >= 2 ** 48 and v not in (16, 17, 10):
                continue                      # 65536^3: the tallest tiles only
            for sk in ((1,) if c else (1, 2, 4, 8, 16, 32)):
                if sk > 1 and words(k) // sk < min_slice_words:
                    continue
                out.append((v, c, sk))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="cost_sweep.jsonl")
    ap.add_argument("--small", action="store_true", help="products below 2^30 bit-operations instead")
    ap.add_argument("--huge", action="store_true", help="the 65536^3 product instead")
    ap.add_argument("--min-slice-words", type=int, default=16)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        sys.exit("cost_sweep needs a GPU")
    import paper_0811_1714_amd as g
    import synth
    g.lib()
    t0 = time.time()
    with open(args.out, "w") as out:
        for (m, k, n) in (small_shapes() if args.small else HUGE_SHAPES if args.huge else SHAPES):
            A = torch.from_numpy(synth.uniform(1, synth.TAG_A, m, k).view(np.int64)).cuda()
            B = torch.from_numpy(synth.uniform(1, synth.TAG_B, k, n).view(np.int64)).cuda()
            C = torch.empty((m, words(n)), dtype=torch.int64, device="cuda")
            lib = g.resolve_schedule(m, k, n)
            reps = 2 if m * k * n >= 2 ** 48 else 3 if m * k * n > 2 ** 42 else (5 if m * k * n > 2 ** 30 else 9)
            for cand in [None] + candidates(m, k, n, args.min_slice_words):
                s = None if cand is None else g.Schedule(g.KERNEL_M4RM, cand[0], cand[1], cand[2])
                ws = g.workspace_bytes(m, k, n, s)
                if ws:
                    g.reserve_workspace(ws)
                for _ in range(2):
                    g.mul(C, A, B, m, k, n, schedule=s)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ts = []
                for _ in range(reps):
                    e0.record()
                    g.mul(C, A, B, m, k, n, schedule=s)
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1))
                rec = {"shape": [m, k, n], "ms": round(float(np.median(ts)), 5)}
                if cand is None:
                    rec["library"] = [lib.variant, lib.cutoff, lib.splitk]
                else:
                    rec.update(variant=cand[0], cutoff=cand[1], splitk=cand[2])
                out.write(json.dumps(rec) + "\n")
            out.flush()
            print(f"{(m, k, n)}: {time.time() - t0:.0f} s", flush=True)
            del A, B, C
            torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
