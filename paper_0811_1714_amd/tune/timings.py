"""Timing dataset for the schedule model: every candidate schedule timed by the library's
autotuner on products with m, k, n log-uniform in [64, 4096) and density log-uniform in
[0.01, 0.5] (the batched workload's shape law).  Columns 0..S-1 of ``*_ms`` are the
isolated latency (gf2_autotune), columns S..2S-1 the per-product time inside a batch of
copies (gf2_autotune_batch).

    python -m paper_0811_1714_amd.tune.timings --count 20000 --heldout 500 --out timings.npz

``--latency-every 4`` times the isolated latency on every fourth training shape only.

A run cut short by ``--budget`` is continued with ``--start <shapes done> --heldout 0``; the
trainer concatenates the training parts of several files.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def shapes(seed, count, tag):
    import synth
    dims = synth.log_uniform_dims(seed, tag, count, 64, 4096)
    dens = synth.log_uniform_p(seed, tag + 1000, count, 0.01, 0.5)
    return dims, dens


def collect(dims, dens, reps, label, budget_s=None, latency_every=1, offset=0):
    """Per-product time inside a batch of copies (gf2_autotune_batch) of every candidate for every
    shape, and the isolated latency (gf2_autotune) for every ``latency_every``-th shape (counted
    from ``offset``; the others keep -1, which the trainer masks out)."""
    import paper_0811_1714_amd as g
    S = g.num_candidates()
    ms = np.full((len(dims), 2 * S), -1.0, dtype=np.float32)
    t0 = time.time()
    done = len(dims)
    for i, ((m, k, n), p) in enumerate(zip(dims, dens)):
        if (offset + i) % latency_every == 0:
            ms[i, :S], _ = g.autotune(int(m), int(k), int(n), float(p), reps)
        ms[i, S:], _, _ = g.autotune_batch(int(m), int(k), int(n), float(p), reps)
        if (i + 1) % 100 == 0:
            print(f"{label}: {i + 1}/{len(dims)} shapes timed, {time.time() - t0:.0f} s", flush=True)
        if budget_s is not None and time.time() - t0 > budget_s:
            done = i + 1
            print(f"{label}: time budget reached after {done} shapes", flush=True)
            break
    return ms[:done], done


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=20000)
    ap.add_argument("--heldout", type=int, default=500)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--budget", type=float, default=None, help="seconds for the training shapes")
    ap.add_argument("--start", type=int, default=0, help="skip this many training shapes (continue a run)")
    ap.add_argument("--latency-every", type=int, default=1,
                    help="time the isolated latency of every n-th training shape only (held-out: all)")
    ap.add_argument("--out", default="timings.npz")
    args = ap.parse_args()
    import paper_0811_1714_amd as g
    g.lib()
    tr_dims, tr_dens = shapes(args.seed, args.count, 11)
    tr_dims, tr_dens = tr_dims[args.start:], tr_dens[args.start:]
    ho_dims, ho_dens = shapes(args.seed, args.heldout, 12)
    ho_ms, _ = collect(ho_dims, ho_dens, args.reps, "held-out")
    tr_ms, n = collect(tr_dims, tr_dens, args.reps, "train", args.budget, args.latency_every, args.start)
    np.savez_compressed(args.out, train_dims=tr_dims[:n], train_density=tr_dens[:n], train_ms=tr_ms,
                        heldout_dims=ho_dims, heldout_density=ho_dens, heldout_ms=ho_ms,
                        candidates=np.array([[c.kernel, c.variant, c.cutoff, c.splitk, c.odd, c.kappa]
                                             for c in (g.candidate(i) for i in range(g.num_candidates()))]))
    print(f"wrote {args.out}: {n} training and {len(ho_dims)} held-out shapes", flush=True)


if __name__ == "__main__":
    main()
