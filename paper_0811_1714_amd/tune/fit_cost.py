"""Fit of the fixed cost model's constants to a ``cost_sweep`` timing file, and the
regret of the schedule it picks per shape.

The model, as the library evaluates it for a schedule (tile, Strassen-Winograd cutoff,
k split) of an m x k by k x n product:

* the recursion halves m, k and n (k and n on word borders) until any dimension is at
  or below the cutoff; each node moves (2mk + 2kn + 2.75mn)/8 bytes in its additions;
* a leaf is cut into row x column tiles (x k slices); a tile of family f costs
  ``tile + phases * (phase + rows * row_phase)``, phases = ceil(k / rows of B per phase);
* tiles run in rounds of one per compute unit; a leaf launch whose last round is at most
  half full spreads that round over all units;
* operand bytes (A once per column tile, B once per row tile), addition bytes, the k
  split's zeroing and its atomic XORs each at a rate of their own.

The fit minimises the log error of the predicted time, weighted six-fold on each shape's
schedules within 15% of its fastest, so the model is sharpest where the choice is made.

    python -m paper_0811_1714_amd.tune.fit_cost paper_0811_1714_amd/tune/cost_sweep_mi355x.jsonl \
        paper_0811_1714_amd/tune/cost_sweep_small_mi355x.jsonl paper_0811_1714_amd/tune/cost_sweep_huge_mi355x.jsonl
"""
import argparse
import collections
import json
import math

import numpy as np

# Tile geometry of the library's M4RM variants: rows, and the tile family (rows of B per
# barrier phase, words of C per row).
TILE_ROWS = {0: 1536, 10: 1408, 1: 1024, 2: 512, 3: 256, 4: 128, 11: 2048, 12: 1024, 13: 512, 14: 1024,
             15: 512, 16: 2048, 17: 1536, 18: 1024}
FAMILY = {0: 16, 10: 16, 1: 16, 2: 16, 3: 16, 4: 16, 11: 64, 12: 64, 13: 64, 14: 256, 15: 256, 16: 32, 17: 32,
          18: 32}
FAMILY_WORDS = {16: 16, 32: 8, 64: 4, 256: 1}
FAMILIES = (16, 32, 64, 256)
CUS = 256
MAX_GROUP = 56


def words(c):
    return (c + 63) // 64


def splittable(m, k, n, cutoff):
    c = max(cutoff, 64)
    return cutoff > 0 and m > c and k > c and n > c


def features(m, k, n, v, cutoff, sk):
    """Per-family counts (tiles, tile-phases, tile-row-phases), byte counts and rounds."""
    acc = {"tiles": 0, "leaves": 0, "op": 0.0, "add": 0.0, "zero": 0.0, "atom": 0.0,
           "t": collections.Counter(), "ph": collections.Counter(), "rph": collections.Counter()}

    def walk(m, k, n, sk):
        if not splittable(m, k, n, cutoff):
            f, bm = FAMILY[v], TILE_ROWS[v]
            rt, ct = -(-m // bm), -(-words(n) // FAMILY_WORDS[f])
            t = rt * ct * sk
            ks = min(k, 64 * (-(-words(k) // sk))) if sk > 1 else k
            ph = -(-ks // f)
            acc["tiles"] += t
            acc["leaves"] += 1
            acc["t"][f] += t
            acc["ph"][f] += t * ph
            acc["rph"][f] += t * ph * bm
            acc["op"] += 8.0 * (m * words(k) * ct + k * words(n) * rt)
            if sk > 1:
                cb = 8.0 * m * words(n)
                acc["zero"] += cb
                acc["atom"] += cb * sk
            return
        acc["add"] += (2.0 * m * k + 2.0 * k * n + 2.75 * m * n) / 8.0
        m0, k0, n0 = (m + 1) // 2, 64 * ((words(k) + 1) // 2), 64 * ((words(n) + 1) // 2)
        for (a, b, c) in [(m0, k0, n0)] * 4 + [(m0, k - k0, n0), (m0, k - k0, n - n0), (m - m0, k - k0, n0)]:
            walk(a, b, c, 1)

    walk(m, k, n, sk)
    full = -(-acc["tiles"] // CUS)
    tail = acc["tiles"] - (full - 1) * CUS
    spread = full >= 2 and 2 * tail <= CUS and 2 <= acc["leaves"] <= MAX_GROUP
    acc["rounds"] = (full - 1) + tail / CUS if spread else full
    return acc


# Parameters: per family (tile us, phase us, row-phase ns), then GB/s of operands,
# additions, zeroing and atomics.
def predict(p, a):
    tile = sum(a["t"][f] * p[3 * i] * 1e-3 + a["ph"][f] * p[3 * i + 1] * 1e-3 + a["rph"][f] * p[3 * i + 2] * 1e-6
               for i, f in enumerate(FAMILIES))
    return (a["rounds"] * tile / a["tiles"] + a["op"] / (p[12] * 1e6) + a["add"] / (p[13] * 1e6)
            + a["zero"] / (p[14] * 1e6) + a["atom"] / (p[15] * 1e6))


def load(*paths):
    rows = [json.loads(line) for path in paths for line in open(path)]
    data = [(tuple(r["shape"]), (r["variant"], r["cutoff"], r["splitk"]), r["ms"]) for r in rows if "library" not in r]
    best = collections.defaultdict(lambda: math.inf)
    for sh, _, ms in data:
        best[sh] = min(best[sh], ms)
    return [(sh, s, ms, features(*sh, *s)) for sh, s, ms in data], best


def fit(data, best, shapes):
    from scipy.optimize import least_squares
    use = [d for d in data if d[0] in shapes]
    w = np.array([6.0 if ms <= 1.15 * best[sh] else 1.0 for sh, _, ms, _ in use])

    def resid(lp):
        p = np.exp(lp)
        return w * np.array([math.log(predict(p, a) / ms) for _, _, ms, a in use])

    p0 = np.log([5.0, 0.6, 0.65] * 4 + [4000, 3000, 3000, 1000])
    return np.exp(least_squares(resid, p0).x)


def regret(data, best, p, shape):
    cands = [(predict(p, a), ms) for sh, _, ms, a in data if sh == shape]
    return min(cands)[1] / best[shape] - 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("sweep", nargs="+")
    ap.add_argument("--cv", action="store_true", help="also leave-one-shape-out regret")
    args = ap.parse_args()
    data, best = load(*args.sweep)
    shapes = list(dict.fromkeys(d[0] for d in data))
    p = fit(data, best, set(shapes))
    for i, f in enumerate(FAMILIES):
        print(f"    {{{f}, {p[3 * i] * 1e-3:.4g}, {p[3 * i + 1] * 1e-3:.4g}, {p[3 * i + 2] * 1e-6:.4g}}},")
    print(f"operands {p[12] * 1e6:.3g} B/ms, additions {p[13] * 1e6:.3g}, zeroing {p[14] * 1e6:.3g}, "
          f"atomics {p[15] * 1e6:.3g}")
    regs = [regret(data, best, p, sh) for sh in shapes]
    for sh, r in zip(shapes, regs):
        print(f"  {sh}: regret {100 * r:.1f}%")
    print(f"in-sample regret: mean {100 * np.mean(regs):.1f}%, max {100 * max(regs):.1f}%")
    if args.cv:
        cv = [regret(data, best, fit(data, best, set(shapes) - {sh}), sh) for sh in shapes]
        print(f"leave-one-shape-out regret: mean {100 * np.mean(cv):.1f}%, max {100 * max(cv):.1f}%")


if __name__ == "__main__":
    main()
