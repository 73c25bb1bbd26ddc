"""Re-time some candidates of a timing set (written by ``tune.timings``) with the current
kernels, after a change to the kernels those candidates run: for every training and held-out
shape, the listed candidates' per-product time inside a batch of copies, and their isolated
latency where the file has latency timings for that shape (``--latency-every`` runs left the
other rows at -1).  The other columns are kept.

    python -m paper_0811_1714_amd.tune.retime --data timings.npz --candidates 7 8 --out new.npz
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def retime(g, dims, dens, ms, cands, reps, label):
    S = g.num_candidates()
    out = ms.copy()
    cols = np.asarray(cands)
    t0 = time.time()
    for i, ((m, k, n), p) in enumerate(zip(dims, dens)):
        b, _ = g.autotune_candidates(int(m), int(k), int(n), cands, float(p), reps, batch=True)
        out[i, S + cols] = b[cols]
        if (ms[i, :S] > 0).any():
            a, _ = g.autotune_candidates(int(m), int(k), int(n), cands, float(p), reps, batch=False)
            out[i, cols] = a[cols]
        if (i + 1) % 200 == 0:
            print(f"{label}: {i + 1}/{len(dims)} shapes re-timed, {time.time() - t0:.0f} s", flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--data", required=True)
    ap.add_argument("--candidates", type=int, nargs="+", required=True)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import paper_0811_1714_amd as g
    g.lib()
    d = dict(np.load(args.data))
    S = g.num_candidates()
    if d["train_ms"].shape[1] != 2 * S:
        raise SystemExit(f"{args.data} has {d['train_ms'].shape[1] // 2} candidates, the library {S}")
    for part in ("heldout", "train"):
        if len(d[f"{part}_dims"]):
            d[f"{part}_ms"] = retime(g, d[f"{part}_dims"], d[f"{part}_density"], d[f"{part}_ms"], args.candidates,
                                     args.reps, part)
    np.savez_compressed(args.out, **d)
    print(f"wrote {args.out}: candidates {args.candidates} re-timed on {len(d['train_dims'])} training and "
          f"{len(d['heldout_dims'])} held-out shapes", flush=True)


if __name__ == "__main__":
    main()
