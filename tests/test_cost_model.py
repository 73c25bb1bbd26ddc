"""The cost model behind the library's default schedule, checked against timings of every
schedule it chooses from (measured on MI355X and stored with the library): the schedule it
picks for each timed shape, and how much slower that is than the fastest."""
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE = os.path.join(ROOT, "paper_0811_1714_amd", "tune")
SWEEPS = [os.path.join(TUNE, f) for f in ("cost_sweep_mi355x.jsonl", "cost_sweep_small_mi355x.jsonl",
                                           "cost_sweep_huge_mi355x.jsonl")]


def timings():
    by = {}
    for line in (line for path in SWEEPS for line in open(path)):
        r = json.loads(line)
        if "library" in r:
            continue
        by.setdefault(tuple(r["shape"]), {})[(r["variant"], r["cutoff"], r["splitk"])] = r["ms"]
    return by


def test_default_schedule_regret_on_timed_shapes():
    import paper_0811_1714_amd as g
    by = timings()
    assert len(by) >= 60
    regret = {}
    for shape, ms in by.items():
        s = g.resolve_schedule(*shape)
        assert s.kernel == g.KERNEL_M4RM
        pick = (s.variant, s.cutoff, s.splitk)
        assert pick in ms, f"{shape}: picked {pick}, which the sweep did not time"
        regret[shape] = ms[pick] / min(ms.values()) - 1
    print({k: round(100 * v, 1) for k, v in regret.items()})
    small = [v for (m, k, n), v in regret.items() if m * k * n < 2 ** 30]
    large = [v for (m, k, n), v in regret.items() if m * k * n >= 2 ** 30]
    assert len(small) >= 40 and np.mean(small) <= 0.03 and max(small) <= 0.15
    assert np.mean(large) <= 0.06 and max(large) <= 0.30
    # The benchmarked squares and rectangles (repeated sweeps differ by about 2-3% per timing).
    for shape in [(8192,) * 3, (16384,) * 3, (32768,) * 3, (65536,) * 3, (10000, 20000, 5000), (4095, 65537, 129)]:
        assert regret[shape] <= 0.03, (shape, regret[shape])
    assert regret[(20001, 777, 30003)] <= 0.10


def test_fit_reproduces_the_library_constants():
    """Refitting the stored sweep gives the constants the library uses: its pick and the
    fit's own argmin agree on every timed shape."""
    import paper_0811_1714_amd as g
    from paper_0811_1714_amd.tune import fit_cost
    data, best = fit_cost.load(*SWEEPS)
    shapes = list(dict.fromkeys(d[0] for d in data))
    p = fit_cost.fit(data, best, set(shapes))
    for shape in shapes:
        cands = [(fit_cost.predict(p, a), s) for sh, s, _, a in data if sh == shape]
        s = g.resolve_schedule(*shape)
        assert min(cands)[1] == (s.variant, s.cutoff, s.splitk), shape
