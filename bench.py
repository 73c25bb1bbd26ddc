"""Benchmark: dense GF(2) products on one MI355X.

One step = one n x n by n x n product over GF(2) (default n = 32768, the
largest square workload), computed by the library's schedule for that shape
(Strassen-Winograd over the M4RM base case), on uniformly random bits
(Bernoulli(1/2), splitmix64-seeded, inputs resident in HBM before timing).

Prints one JSON line.  ``value`` is effective bit-operations per second,
2*n^3 / (seconds per product) -- one AND and one XOR per inner-product term.
``roofline`` reports the dominant kernel (the launch of all M4RM leaves), timed
live with HIP event pairs the library records around each of its launches, as
64-bit table-row additions (table builds included) against the VALU peak; beside
it the whole product against its roof (leaves at the VALU peak plus the
Strassen-Winograd passes at the HBM peak) and the leaf launch's LDS traffic
against the LDS rates the library's probe kernels measure in the same run.
``batch`` times 4096 log-uniform products batched (fixed and learned schedules)
against the plain form.  ``cpu_baseline`` times the CPU oracle, built for this
host, on bounded samples of rows of the same product at 1 and at all threads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_WORD_XOR_PEAK = 256 * 64 * 2.4e9   # 64-bit table-row additions/s: 256 CUs x 64 lanes x 2.4 GHz, one
                                          # v_bitop3 on a 32-bit half folds two table words into the sum
HBM_PEAK = 8.0e12                         # bytes/s
LDS_NOMINAL = 256 * 2.4e9 * 256           # bytes/s: 64 banks x 4 B per clock, 256 CUs, 2.4 GHz (reference only)
MFMA_I8_PEAK = 5.0e15                     # int8 dense matrix-core ops/s (one multiply-accumulate = 2 ops)
BUILD_BYTES = 256 * 64 * 4                # LDS bytes stored per table build: 256 entries x 64 B x 4 tables (= 64 KiB
                                          # for every tile family: t tables x 256 entries x tile width)
BUILD_XORS = 255 * 32                     # 64-bit XORs per build: 255 entries x (t x tile words = 32)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--kernel", choices=["m4rm", "mfma"], default="m4rm",
                    help="base case of the timed product (mfma: the int8 matrix-core parity kernel)")
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--cutoff", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--sweep", action="store_true", help="time candidate schedules for n = 8K, 16K, 32K")
    ap.add_argument("--sweep-n", type=int, nargs="*", default=None)
    ap.add_argument("--sweep-variants", type=int, nargs="*", default=None)
    ap.add_argument("--copy-calibration", action="store_true", help="run a plain 1 GiB device copy (counter scale)")
    ap.add_argument("--lds-calibration", action="store_true",
                    help="measure LDS read and write bandwidth with the library's probe kernels")
    ap.add_argument("--batch", type=int, default=4096,
                    help="also time a batch of this many log-uniform products (0: skip)")
    ap.add_argument("--rect", action="store_true", help="time the rectangular and ragged products (library schedule)")
    ap.add_argument("--ablation", action="store_true",
                    help="base-case variants of Section 3 at equal size: one table per stripe, t = 2, t = 8")
    ap.add_argument("--narrow", action="store_true", help="matrix-vector and narrow-B products against the HBM roof")
    ap.add_argument("--configs", action="store_true",
                    help="1024^3 plain M4RM, and 8K/16K/32K on the library schedule and on the int8 matrix-core base")
    ap.add_argument("--odd-sweep", action="store_true",
                    help="padding vs peeling around 2^14 and at word-misaligned sizes")
    return ap.parse_args()


def default_schedule(g, n):
    """The schedule the library itself runs for an n x n product under its default policy (the
    cost model's choice; at n = 32768: two Strassen-Winograd levels over the four-table M4RM
    tile of 2048 rows x 512 columns)."""
    pol = g.get_policy()
    g.set_policy(g.POLICY_FIXED)
    try:
        return g.resolve_schedule(n, n, n)
    finally:
        g.set_policy(pol)


def m4rm_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_0811_1714_amd", "csrc", "m4rm.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def traffic_from_profile(n, sched):
    """HBM bytes per M4RM launch from the committed rocprofv3 counter summary, or None when
    the summary is for another kernel source, workload or schedule."""
    path = os.path.join(ROOT, "profiles", "m4rm_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if (rec.get("m4rm_source_sha256_16") != m4rm_source_hash() or rec.get("n") != n
            or rec.get("variant") != sched.variant or rec.get("cutoff") != sched.cutoff):
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_calibration():
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


def lds_calibration(g, quiet=False):
    """LDS bandwidth of the probe kernels (reads as the lookups issue them, writes as the table
    build issues them), timed with HIP events on the launch stream: the measured ceiling for
    the M4RM kernels' table traffic."""
    import torch
    blocks = 8 * 256
    out = torch.empty(blocks * 1024, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    res = {}
    for mode, name, iters in ((0, "read_b128", 64), (1, "write_b32", 256)):
        for _ in range(2):
            g.lds_probe(mode, blocks, iters, out, stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        times = []
        for _ in range(5):
            e0.record(stream)
            nbytes = g.lds_probe(mode, blocks, iters, out, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        res[name] = {"bytes": nbytes, "ms": ms, "bytes_per_s": nbytes / (ms * 1e-3),
                     "bytes_per_clk_per_cu_at_2.4GHz": nbytes / (ms * 1e-3) / (256 * 2.4e9)}
    if not quiet:
        print(json.dumps({"lds_calibration": res}), flush=True)
    return res


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def time_product(g, dA, dB, dC, n, sched, steps, warmup):
    import torch
    for _ in range(warmup):
        g.mul(dC, dA, dB, n, n, n, schedule=sched)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for i in range(steps):
        g.mul(dC, dA, dB, n, n, n, schedule=sched)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    total = evs[0].elapsed_time(evs[-1])
    return total / steps, per


SWEEP_N = (8192, 16384, 32768)
SWEEP_VARIANTS = None


def sweep(g):
    import torch
    import synth
    for n in SWEEP_N:
        A = synth.uniform(1, synth.TAG_A, n, n)
        B = synth.uniform(1, synth.TAG_B, n, n)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.empty_like(dA)
        for cutoff in (0, n // 2, n // 4, n // 8):
            if cutoff and cutoff < 2048:
                continue
            for v in SWEEP_VARIANTS or range(g.kernel_variants(g.KERNEL_M4RM)):
                s = g.Schedule(g.KERNEL_M4RM, v, cutoff, 1)
                ms, per = time_product(g, dA, dB, dC, n, s, 3, 1)
                print(json.dumps({"n": n, "variant": v, "cutoff": cutoff, "ms": round(min(per), 4),
                                  "eff_bitops": 2 * n ** 3 / (min(per) * 1e-3)}), flush=True)
        del dA, dB, dC
        torch.cuda.empty_cache()


def configs_bench(g):
    """Config 1 (1024^3, M4RM with 8-bit tables, no Strassen: every 16-wave tile height) and
    config 2 (n = 8192, 16384, 32768: the library's schedule, the same recursion over the int8
    matrix-core base, and that base without recursion).  Median of 10, HIP events."""
    import torch
    import synth

    def med(dA, dB, dC, n, s, reps=10):
        ws = g.workspace_bytes(n, n, n, s) if s is not None else 0
        if ws:
            g.reserve_workspace(ws)
        for _ in range(2):
            g.mul(dC, dA, dB, n, n, n, schedule=s)
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        evs[0].record()
        for i in range(reps):
            g.mul(dC, dA, dB, n, n, n, schedule=s)
            evs[i + 1].record()
        torch.cuda.synchronize()
        per = [evs[i].elapsed_time(evs[i + 1]) for i in range(reps)]
        return float(np.median(per)), float(np.mean(per))

    A = synth.uniform(0, synth.TAG_A, 1024, 1024)
    B = synth.uniform(0, synth.TAG_B, 1024, 1024)
    dA, dB = to_dev(A), to_dev(B)
    dC = torch.empty_like(dA)
    for v in (0, 10, 1, 2, 3, 4, 11, 12, 13, 14, 15, 16, 17, 18):
        ms, mean = med(dA, dB, dC, 1024, g.Schedule(g.KERNEL_M4RM, v, 0, 1))
        print(json.dumps({"config": 1, "n": 1024, "schedule": {"kernel": "m4rm", "variant": v}, "ms": round(ms, 4),
                          "mean_ms": round(mean, 4), "eff_bitops": 2 * 1024 ** 3 / (ms * 1e-3)}), flush=True)
    lib = g.resolve_schedule(1024, 1024, 1024)
    ms, mean = med(dA, dB, dC, 1024, lib)
    print(json.dumps({"config": 1, "n": 1024, "schedule": "library", "variant": lib.variant, "splitk": lib.splitk,
                      "ms": round(ms, 4), "mean_ms": round(mean, 4), "eff_bitops": 2 * 1024 ** 3 / (ms * 1e-3)}),
          flush=True)
    for n in (8192, 16384, 32768):
        A = synth.uniform(1, synth.TAG_A, n, n)
        B = synth.uniform(1, synth.TAG_B, n, n)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.empty_like(dA)
        lib = g.resolve_schedule(n, n, n)
        runs = [("library", lib), ("mfma-base", g.Schedule(g.KERNEL_MFMA, 0, lib.cutoff, 1)),
                ("mfma-base, no recursion", g.Schedule(g.KERNEL_MFMA, 0, 0, 1))]
        for name, s in runs:
            ms, mean = med(dA, dB, dC, n, s, reps=5 if n == 32768 else 10)
            print(json.dumps({"config": 2, "n": n, "schedule": name, "kernel": s.kernel, "variant": s.variant,
                              "cutoff": s.cutoff, "splitk": s.splitk, "ms": round(ms, 4), "mean_ms": round(mean, 4),
                              "eff_bitops": 2 * n ** 3 / (ms * 1e-3)}), flush=True)
        del dA, dB, dC
        torch.cuda.empty_cache()


ABLATION = ((21, "one table per 8-row stripe for all m rows, C in global memory (Alg. 1), 512 x 512 blocks"),
            (5, "one table per 8-row stripe (Alg. 2), 768 x 2048"), (6, "one table, 512 x 2048"),
            (0, "t = 2 (Alg. 3), 1536 x 1024"), (10, "t = 2, 1408 x 1024"), (1, "t = 2, 1024 x 1024"),
            (2, "t = 2, 512 x 1024"), (11, "t = 8 (Alg. 3), 2048 x 256"), (12, "t = 8, 1024 x 256"),
            (13, "t = 8, 512 x 256"), (22, "t = 8, 4096 x 256"), (16, "t = 4 (Alg. 3), 2048 x 512"), (17, "t = 4, 1536 x 512"),
            (18, "t = 4, 1024 x 512"))


def ablation_bench(g):
    """Section 3's base-case variants on the GPU at equal size: an n x n product with no
    Strassen recursion, every tile organisation, 8-bit tables (kappa = 8) throughout."""
    import torch
    import synth
    for n in (8192, 16384):
        A = synth.uniform(1, synth.TAG_A, n, n)
        B = synth.uniform(1, synth.TAG_B, n, n)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.empty_like(dA)
        for v, name in ABLATION:
            if v == 21 and n > 8192:
                # Alg. 1 reads and rewrites C in global memory once per 8-row stripe: m * k/8 * n/64 * 16
                # bytes (137 GB at n = 16384), seconds per product; n = 8192 shows the comparison.
                continue
            s = g.Schedule(g.KERNEL_M4RM, v, 0, 1)
            ms, per = time_product(g, dA, dB, dC, n, s, 3 if v == 21 else 5, 1 if v == 21 else 2)
            wx = n * (n // 8) * (n // 64)
            print(json.dumps({"n": n, "variant": v, "tile": name, "ms": round(float(np.median(per)), 4),
                              "table_row_additions_per_s": wx / (float(np.median(per)) * 1e-3)}), flush=True)
        del dA, dB, dC
        torch.cuda.empty_cache()


NARROW = ((32768, 32768, 1), (32768, 32768, 8), (32768, 32768, 64), (32768, 32768, 129), (32768, 32768, 256),
          (4095, 65537, 129), (4095, 65537, 64))


def narrow_bench(g):
    """Matrix-vector and narrow-B products: the popcount kernel (A read once), the eight-table
    M4RM tile with a k split, the library's choice and the int8 matrix core, against the HBM roof
    (A + B + C once at 8 TB/s)."""
    import torch
    import synth
    for (m, k, n) in NARROW:
        A = synth.uniform(1, synth.TAG_A, m, k)
        B = synth.uniform(1, synth.TAG_B, k, n)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.empty((m, (n + 63) // 64), dtype=torch.int64, device="cuda")
        hbm = 8.0 * (m * ((k + 63) // 64) + k * ((n + 63) // 64) + m * ((n + 63) // 64))
        lib = g.resolve_schedule(m, k, n)
        for name, s in (("library", None), ("popcount", g.Schedule(g.KERNEL_CUBIC, 0, 0, 1)),
                        ("eight-table, k/32", g.Schedule(g.KERNEL_M4RM, 13, 0, 32)),
                        ("int8 matrix core", g.Schedule(g.KERNEL_MFMA, 0, 0, 1))):
            ws = g.workspace_bytes(m, k, n, s) if s is not None else 0
            if ws:
                g.reserve_workspace(ws)
            for _ in range(2):
                g.mul(dC, dA, dB, m, k, n, schedule=s)
            torch.cuda.synchronize()
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
            evs[0].record()
            for i in range(10):
                g.mul(dC, dA, dB, m, k, n, schedule=s)
                evs[i + 1].record()
            torch.cuda.synchronize()
            ms = float(np.median([evs[i].elapsed_time(evs[i + 1]) for i in range(10)]))
            print(json.dumps({"m": m, "k": k, "n": n, "schedule": name,
                              "resolved": None if s is not None else [lib.kernel, lib.variant, lib.cutoff, lib.splitk],
                              "ms": round(ms, 4), "hbm_roof_ms": round(hbm / 8e12 * 1e3, 4),
                              "hbm_frac": round(hbm / 8e12 * 1e3 / ms, 3)}), flush=True)
        del dA, dB, dC
        torch.cuda.empty_cache()


RECT_SHAPES = ((10000, 20000, 5000), (20001, 777, 30003), (4095, 65537, 129))


def rect_bench(g):
    """The rectangular and ragged products at p = 1/2 and p = 0.01 (stored dense) under the
    library's own schedule, and the int8 matrix-core base for comparison.  Compulsory HBM
    bytes = A + B + C once."""
    import torch
    import synth
    for (m, k, n) in RECT_SHAPES:
        for p in (0.5, 0.01):
            A = synth.bernoulli(1, synth.TAG_A, m, k, p)
            B = synth.bernoulli(1, synth.TAG_B, k, n, p)
            dA, dB = to_dev(A), to_dev(B)
            dC = torch.empty((m, (n + 63) // 64), dtype=torch.int64, device="cuda")
            hbm = 8.0 * (m * ((k + 63) // 64) + k * ((n + 63) // 64) + m * ((n + 63) // 64))
            for name, sched in (("library", None), ("mfma", g.Schedule(g.KERNEL_MFMA, 0, 0, 1))):
                for _ in range(2):
                    g.mul(dC, dA, dB, m, k, n, schedule=sched)
                torch.cuda.synchronize()
                evs = [torch.cuda.Event(enable_timing=True) for _ in range(11)]
                evs[0].record()
                for i in range(10):
                    g.mul(dC, dA, dB, m, k, n, schedule=sched)
                    evs[i + 1].record()
                torch.cuda.synchronize()
                per = [evs[i].elapsed_time(evs[i + 1]) for i in range(10)]
                ms = float(np.median(per))
                print(json.dumps({"m": m, "k": k, "n": n, "p": p, "schedule": name, "ms": round(ms, 4),
                                  "eff_bitops": 2.0 * m * k * n / (ms * 1e-3),
                                  "hbm_compulsory_bytes": hbm, "hbm_roof_ms": hbm / 8e12 * 1e3,
                                  "word_xors": m * ((k + 7) // 8) * ((n + 63) // 64),
                                  "valu_roof_ms": m * ((k + 7) // 8) * ((n + 63) // 64) / VALU_WORD_XOR_PEAK * 1e3}),
                      flush=True)
            del dA, dB, dC
            torch.cuda.empty_cache()


ODD_SIZES = (16383, 16384, 16385, 16320, 16448, 16000)


def odd_sweep(g):
    """Odd sizes in Strassen-Winograd: virtual zero padding against peeling, n x n products
    around 2^14 and at sizes that are not multiples of 128.  Two levels for every size (the
    cutoff n/4 + 128 stops both rules after two halvings), the headline's 2048 x 512 tiles."""
    import torch
    import synth
    for n in ODD_SIZES:
        A = synth.uniform(1, synth.TAG_A, n, n)
        B = synth.uniform(1, synth.TAG_B, n, n)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.empty_like(dA)
        outs = {}
        for odd, name in ((g.ODD_PAD, "pad"), (g.ODD_PEEL, "peel")):
            s = g.Schedule(g.KERNEL_M4RM, 16, n // 4 + 128, 1, odd)
            ws = g.workspace_bytes(n, n, n, s)
            if ws:
                g.reserve_workspace(ws)
            ms, per = time_product(g, dA, dB, dC, n, s, 5, 2)
            outs[name] = dC.clone()
            print(json.dumps({"n": n, "odd": name, "cutoff": s.cutoff, "ms": round(float(np.median(per)), 4),
                              "eff_bitops": 2 * n ** 3 / (float(np.median(per)) * 1e-3),
                              "workspace_bytes": ws}), flush=True)
        assert torch.equal(outs["pad"], outs["peel"]), f"n={n}: peeling and padding differ"
        del dA, dB, dC, outs
        torch.cuda.empty_cache()


def batch_bench(g, count, steps, warmup, seed=3, lo=64, hi=4096):
    """Config 4: ``count`` independent products, m, k, n log-uniform in [lo, hi) (Bernoulli(1/2)
    bits generated on the device).  Times the persistent graph-captured batch against the plain
    form (one gf2_mul per product, fixed default schedule)."""
    import torch
    import synth
    dims = synth.log_uniform_dims(seed, 4, count, lo, hi)
    W = lambda c: (int(c) + 63) // 64
    sizes = [int(m) * W(k) + int(k) * W(n) + int(m) * W(n) for m, k, n in dims]
    offs = np.concatenate([[0], np.cumsum([(s + 31) // 32 * 32 for s in sizes])])
    gen = torch.Generator(device="cuda").manual_seed(seed)
    pool = torch.randint(-(1 << 62), 1 << 62, (int(offs[-1]),), dtype=torch.int64, device="cuda", generator=gen)
    probs = []
    for i, (m, k, n) in enumerate(dims):
        m, k, n = int(m), int(k), int(n)
        base = int(offs[i])
        A = pool[base: base + m * W(k)].view(m, W(k))
        B = pool[base + m * W(k): base + m * W(k) + k * W(n)].view(k, W(n))
        C = pool[base + m * W(k) + k * W(n): base + sizes[i]].view(m, W(n))
        probs.append((C, A, B, m, k, n))
    plist = [g.problem(C, A, B, m, k, n) for (C, A, B, m, k, n) in probs]
    total_ops = float(sum(2.0 * m * k * n for (_, _, _, m, k, n) in probs))
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"count": count, "total_bitops": total_ops, "pool_bytes": int(offs[-1]) * 8}
    g.set_policy(g.POLICY_FIXED)
    out["ms_plain"] = timed(lambda: [g.mul(C, A, B, m, k, n) for (C, A, B, m, k, n) in probs], max(1, steps // 2))
    out["ms_batched_fixed"] = timed(lambda: g.mul_batched(plist), steps)
    if os.path.exists(g.DEFAULT_MODEL):
        g.load_model()
        g.set_policy(g.POLICY_MODEL)
        out["ms_batched_model"] = timed(lambda: g.mul_batched(plist), steps)
        plan = g.BatchPlan(plist)
        out["model_schedule_histogram"] = np.bincount([plan.schedule(i) for i in range(count)],
                                                      minlength=g.num_candidates()).tolist()
        plan.destroy()
        g.set_policy(g.POLICY_FIXED)
        g.set_model(None)
    best = min(v for kk, v in out.items() if kk.startswith("ms_batched"))
    out["bitops_batched_best"] = total_ops / (best * 1e-3)
    out["bitops_plain"] = total_ops / (out["ms_plain"] * 1e-3)
    out["speedup_vs_plain"] = out["ms_plain"] / best
    if "ms_batched_model" in out:
        out["model_gain_vs_fixed"] = out["ms_batched_fixed"] / out["ms_batched_model"]
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, C, n, seconds):
    """The oracle (row-by-row packed XOR, Sections 1 and 2) on bounded samples of rows of the same
    product, timed on this host: first at one thread, then at every thread OpenMP is given, each
    about ``seconds / 2`` of CPU time.  The oracle is compiled here with -O3 -march=native (the
    in-tree build is generic x86-64).  The rows it computes are compared with those rows of the
    GPU's product ``C`` (host copy).  Returns (baseline record, rows bit-exact)."""
    import tempfile
    import oracle
    from oracle import build as obuild
    build_dir = tempfile.mkdtemp(prefix="gf2ref_native_")
    try:
        oracle.use_library(obuild.build(native=True, out_dir=build_dir))
        flags = obuild.command(native=True)
    except Exception as e:                      # no compiler on this host: the in-tree -O3 build
        oracle.use_library(None)
        flags = obuild.command(native=False) + f" (native build failed: {type(e).__name__})"

    def timed(threads, budget):
        rows = 4
        t0 = time.perf_counter()
        oracle.mul_rows(A, B, n, n, n, np.arange(rows), nthreads=threads)
        dt = time.perf_counter() - t0
        rows = int(max(4, min(n, rows * budget / max(dt, 1e-6))))
        sel = np.arange(rows) * (n // rows)
        t0 = time.perf_counter()
        ref = oracle.mul_rows(A, B, n, n, n, sel, nthreads=threads)
        dt = time.perf_counter() - t0
        return rows, dt, bool(np.array_equal(C[sel], ref))

    threads = oracle.max_threads()
    r1, dt1, ok1 = timed(1, seconds / 2)
    rn, dtn, okn = timed(threads, seconds / 2)
    oracle.use_library(None)
    exact = ok1 and okn
    rec = {"value": 2.0 * rn * n * n / dtn, "unit": "bit-ops/s", "cores": threads, "kind": "oracle",
           "sample": f"{rn} of {n} rows of the n={n} product at {threads} threads ({dtn:.1f} s) and {r1} rows at "
                     f"1 thread ({dt1:.1f} s), row-by-row packed XOR; the same rows of the GPU product compared: "
                     f"{'bit-exact' if exact else 'DIFFERENT'}",
           "single_thread": {"value": 2.0 * r1 * n * n / dt1, "unit": "bit-ops/s", "cores": 1},
           "cpu_model": cpu_model(), "build": flags}
    return rec, exact


def table_builds(n, sched):
    """Table builds (one per barrier phase per tile, 64 KiB of LDS stores and 8160 64-bit XORs
    each) in the M4RM leaves of an n x n product under ``sched``; None for tiles the cost
    model does not describe."""
    from paper_0811_1714_amd.tune import fit_cost
    if sched.variant not in fit_cost.FAMILY:
        return None
    acc = fit_cost.features(n, n, n, sched.variant, sched.cutoff, max(1, sched.splitk))
    return sum(acc["ph"].values())


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_0811_1714_amd as g
    import synth

    g.lib()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.lds_calibration:
        lds_calibration(g)
        return
    if args.odd_sweep:
        odd_sweep(g)
        return
    if args.rect:
        rect_bench(g)
        return
    if args.configs:
        configs_bench(g)
        return
    if args.ablation:
        ablation_bench(g)
        return
    if args.narrow:
        narrow_bench(g)
        return
    if args.sweep:
        global SWEEP_N, SWEEP_VARIANTS
        if args.sweep_n:
            SWEEP_N = tuple(args.sweep_n)
        SWEEP_VARIANTS = args.sweep_variants
        sweep(g)
        return
    n = args.n
    sched = default_schedule(g, n)
    if args.kernel == "mfma":
        sched = g.Schedule(g.KERNEL_MFMA, 0, 0, 1)
    if args.variant is not None:
        sched.variant = args.variant
    if args.cutoff is not None:
        sched.cutoff = args.cutoff
    A = synth.uniform(1, synth.TAG_A, n, n)
    B = synth.uniform(1, synth.TAG_B, n, n)
    dA, dB = to_dev(A), to_dev(B)
    dC = torch.empty_like(dA)
    ws = g.workspace_bytes(n, n, n, sched)
    if ws:
        g.reserve_workspace(ws)

    for _ in range(args.warmup):
        g.mul(dC, dA, dB, n, n, n, schedule=sched)
    torch.cuda.synchronize()
    g.trace_clear()
    g.trace_enable(True)
    ms, per = time_product(g, dA, dB, dC, n, sched, args.steps, 0)
    g.trace_enable(False)
    recs = g.trace_read()
    g.trace_clear()

    C = dC.cpu().numpy().view(np.uint64)    # the timed product; the CPU leg compares rows of it

    # Workspace of the timed (breadth-first) plan, and of the same schedule with Section 4's
    # two-temporary form at the top level, timed too and compared with the timed product.
    workspace = {"bytes": ws, "operand_bytes": 3 * n * ((n + 63) // 64) * 8}
    if args.kernel == "m4rm" and sched.cutoff:
        low = g.Schedule(sched.kernel, sched.variant, sched.cutoff, sched.splitk, sched.odd, sched.kappa, g.MEM_LOW)
        fast_c = dC.clone()
        low_ms, _ = time_product(g, dA, dB, dC, n, low, max(3, args.steps // 2), 2)
        workspace["two_temporary"] = {"bytes": g.workspace_bytes(n, n, n, low), "ms_per_step": low_ms,
                                      "same_bits": bool(torch.equal(fast_c, dC))}
        del fast_c

    if args.kernel == "mfma":
        mf = [r for r in recs if r[0] == "mfma"]
        launches = len(mf)
        work = sum(r[2] for r in mf) / max(1, launches)      # multiply-accumulates per launch
        kms = sum(r[3] for r in mf) / max(1, launches)
        roofline = {"bound": "mfma", "kernel": "int8 matrix-core base", "achieved": 2.0 * work / (kms * 1e-3) / 1e12,
                    "peak": MFMA_I8_PEAK / 1e12, "unit": "TOP/s", "frac": 2.0 * work / (kms * 1e-3) / MFMA_I8_PEAK,
                    "traffic": None, "launches_per_step": launches / max(1, args.steps), "kernel_ms": kms,
                    "macs_per_launch": work}
    else:
        m4 = [r for r in recs if r[0] == "m4rm"]
        launches = len(m4)
        work = sum(r[2] for r in m4) / max(1, launches)      # 64-bit table-row additions per launch
        kms = sum(r[3] for r in m4) / max(1, launches)
        # One table build per barrier phase per tile: 8160 64-bit XORs and 64 KiB of LDS stores.
        builds = table_builds(n, sched)
        builds = builds * args.steps / max(1, launches) if builds is not None else 0.0
        xors = work + BUILD_XORS * builds
        achieved = xors / (kms * 1e-3)
        # Whole product against its roof: every leaf's word-XORs (builds included) at the VALU
        # peak plus the bytes the Strassen-Winograd passes and zero fills move at the HBM peak.
        pass_bytes = sum(r[2] for r in recs if r[0] in ("strassen_pre", "strassen_post", "fill")) / args.steps
        t_roof = (xors * launches / args.steps) / VALU_WORD_XOR_PEAK + pass_bytes / HBM_PEAK
        # LDS, the unit that binds in practice: lookups read 8 B per table-row addition, builds
        # store 64 KiB each; against the read and write rates the probe kernels measure.
        lds = lds_calibration(g, quiet=True)
        rd, wr = lds["read_b128"]["bytes_per_s"], lds["write_b32"]["bytes_per_s"]
        lookup_bytes, build_bytes = 8.0 * work, BUILD_BYTES * builds
        t_lds = lookup_bytes / rd + build_bytes / wr
        roofline = {"bound": "alu", "kernel": "m4rm leaves (all Strassen-Winograd leaves in one launch)",
                    "achieved": achieved / 1e12, "peak": VALU_WORD_XOR_PEAK / 1e12, "unit": "T word-XOR/s",
                    "frac": achieved / VALU_WORD_XOR_PEAK, "traffic": traffic_from_profile(n, sched),
                    "launches_per_step": launches / max(1, args.steps), "kernel_ms": kms,
                    "word_xors_per_launch": work, "table_builds_per_launch": builds,
                    "build_xors_per_launch": BUILD_XORS * builds,
                    "product": {"roof_ms": t_roof * 1e3, "frac": t_roof * 1e3 / ms,
                                "strassen_and_fill_bytes": pass_bytes},
                    "fixed_reference": {"what": "kappa=8 M4RM without recursion at the VALU peak",
                                        "roof_ms": n * ((n + 7) // 8) * ((n + 63) // 64) / VALU_WORD_XOR_PEAK * 1e3,
                                        "frac": n * ((n + 7) // 8) * ((n + 63) // 64) / VALU_WORD_XOR_PEAK * 1e3 / ms},
                    "lds": {"lookup_bytes_per_launch": lookup_bytes, "build_bytes_per_launch": build_bytes,
                            "read_peak_measured": rd, "write_peak_measured": wr,
                            "roof_ms": t_lds * 1e3, "frac": t_lds * 1e3 / kms,
                            "frac_of_nominal_read_peak": (lookup_bytes + build_bytes) / (kms * 1e-3) / LDS_NOMINAL}}
    out = {
        "metric": "ms and effective GF(2) bit-ops/s per n x n product, % roofline",
        "value": 2.0 * n ** 3 / (ms * 1e-3),
        "unit": "bit-ops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 (bit-packed GF(2))" if args.kernel == "m4rm" else "i8 (0/1 entries, int32 sums)",
        "data": "synthetic",
        "config": {"workload": f"square GF(2) product n={n}, Bernoulli(1/2) bits, packed 64 per word",
                   "n": n, "schedule": {"kernel": args.kernel, "variant": sched.variant, "cutoff": sched.cutoff,
                                        "splitk": sched.splitk},
                   "ms_min": min(per), "ms_median": float(np.median(per)), "bit_exact_sampled_rows": None},
        "roofline": roofline,
        "workspace": workspace,
    }
    if args.batch:
        del dA, dB, dC
        torch.cuda.empty_cache()
        out["batch"] = batch_bench(g, args.batch, max(3, args.steps), 1)
    exact = None
    if not args.no_cpu:
        out["cpu_baseline"], exact = cpu_baseline(A, B, C, n, args.cpu_seconds)
        out["config"]["bit_exact_sampled_rows"] = exact
    print(json.dumps(out), flush=True)
    if exact is False:
        sys.exit(1)


if __name__ == "__main__":
    main()
