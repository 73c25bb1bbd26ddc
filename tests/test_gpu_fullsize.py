"""GPU parity at the full workload sizes, in the launch configurations the benchmark times.

At these sizes the oracle cannot produce whole products in seconds, so each result is checked
two ways:

* sampled rows (first, last and evenly spaced ones) against the oracle's row-by-row product,
  bit for bit;
* every row through Freivalds' test with 64 random vectors at once: C.X must equal A.(B.X)
  for a random n x 64 matrix X.  A wrong C passes with probability at most 2^-64, and the
  three products involved are cheap for the oracle (one output word per row).

Inputs are the seeded Bernoulli streams used everywhere else.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
import synth
from gf2_testutil import SENTINEL, from_dev, operand, to_dev

TAG_FREIVALDS = 3


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    return g


def sample_rows(m, count=64):
    return np.unique(np.concatenate([[0, m - 1], np.linspace(0, m - 1, count).astype(np.int64)]))


def check_full(A, B, C, m, k, n, label):
    W = (n + 63) // 64
    rows = sample_rows(m)
    ref = oracle.mul_rows(A, B, m, k, n, rows)
    assert np.array_equal(C[rows, :W], ref), f"{label}: sampled rows differ from the oracle"
    X = synth.uniform(17, TAG_FREIVALDS, n, 64)
    CX = oracle.mul(C[:, :W], X, m, n, 64)
    ABX = oracle.mul(A, oracle.mul(B, X, k, n, 64), m, k, 64)
    assert np.array_equal(CX, ABX), f"{label}: Freivalds test failed (some row of C is wrong)"
    if n % 64:
        assert not np.any(C[:, W - 1] >> np.uint64(n % 64)), f"{label}: padding bits of C not zero"


def run(g, A, B, m, k, n, schedule, ldc_pad=1):
    import torch
    W = (n + 63) // 64
    dA, dB = to_dev(A), to_dev(B)
    C0 = np.full((m, W + ldc_pad), SENTINEL, dtype=np.uint64)
    dC = to_dev(C0)
    if schedule is not None:
        ws = g.workspace_bytes(m, k, n, schedule)
        if ws:
            g.reserve_workspace(ws)
    g.mul(dC, dA, dB, m, k, n, schedule=schedule)
    torch.cuda.synchronize()
    C = from_dev(dC)
    del dA, dB, dC
    assert np.all(C[:, W:] == SENTINEL), "stride-gap words of C were written"
    return C


@pytest.mark.parametrize("n", [8192, 16384, 32768])
def test_square_products_as_benchmarked(g, n):
    """n x n by n x n, Bernoulli(1/2): the benchmark's schedule (Strassen-Winograd, cutoff n/4, over
    the M4RM base case), the int8 matrix-core base under the same recursion, and the library's
    own choice."""
    import bench
    A = synth.uniform(1, synth.TAG_A, n, n)
    B = synth.uniform(1, synth.TAG_B, n, n)
    scheds = {"bench": bench.default_schedule(g, n),
              "mfma-base": g.Schedule(g.KERNEL_MFMA, 0, n // 4, 1),
              "library": None}
    first = None
    for name, s in scheds.items():
        print(f"n={n} schedule {name}", flush=True)
        C = run(g, A, B, n, n, n, s, ldc_pad=0)
        if first is None:
            check_full(A, B, C, n, n, n, f"{n}^3 {name}")
            first = C
        else:
            assert np.array_equal(C, first), f"{n}^3 {name}: bits differ from the benchmark schedule"


def test_leaf_launch_with_k_split_tail(g):
    """A Strassen leaf launch whose last round of tiles would be half empty cuts its last
    leaves into k slices XOR-ed atomically into their zeroed results (8192 x 4096 x 8192,
    one level, 128-row tiles: 896 tiles on 256 compute units).  Also at two levels with
    1408-row tiles and odd sizes (294 tiles), with 2048 x 512 four-table tiles (588 tiles),
    and in accumulate mode."""
    for (m, k, n, v, cutoff, acc) in [(8192, 4096, 8192, 4, 2048, False), (10001, 5000, 9000, 10, 2314, False),
                                      (12000, 6000, 12000, 16, 3000, False), (8192, 4096, 8192, 4, 2048, True)]:
        print(f"tail split {(m, k, n)} variant {v} cutoff {cutoff} accumulate {acc}", flush=True)
        A = synth.uniform(21, synth.TAG_A, m, k)
        B = synth.uniform(21, synth.TAG_B, k, n)
        s = g.Schedule(g.KERNEL_M4RM, v, cutoff, 1)
        if not acc:
            C = run(g, A, B, m, k, n, s)
            check_full(A, B, C, m, k, n, f"tail split {(m, k, n)}")
        else:
            import torch
            W = (n + 63) // 64
            C0 = synth.uniform(22, synth.TAG_C, m, n)
            dC = to_dev(C0)
            g.reserve_workspace(g.workspace_bytes(m, k, n, s))
            g.mul(dC, to_dev(A), to_dev(B), m, k, n, accumulate=True, schedule=s)
            torch.cuda.synchronize()
            rows = sample_rows(m)
            got = from_dev(dC)[rows, :W]
            assert np.array_equal(got, C0[rows, :W] ^ oracle.mul_rows(A, B, m, k, n, rows)), "addmul differs"


RECT = [(10000, 20000, 5000), (20001, 777, 30003), (4095, 65537, 129)]


@pytest.mark.parametrize("p", [0.5, 0.01])
@pytest.mark.parametrize("m,k,n", RECT)
def test_rectangular_ragged_full_size(g, m, k, n, p):
    """The rectangular and ragged products, dense and sparse bits stored dense, with garbage in
    the inputs' padding; library schedule and the int8 matrix-core base."""
    seed = 1000 + RECT.index((m, k, n))
    print(f"rect {(m, k, n)} p={p} generating", flush=True)
    A = operand(seed, synth.TAG_A, m, k, ld=(k + 63) // 64 + 1, garbage=True, p=p)
    B = operand(seed, synth.TAG_B, k, n, ld=(n + 63) // 64, garbage=True, p=p)
    first = None
    for name, s in (("library", None), ("mfma-base", g.Schedule(g.KERNEL_MFMA, 0, 0, 1))):
        print(f"rect {(m, k, n)} p={p} schedule {name}", flush=True)
        C = run(g, A, B, m, k, n, s)
        if first is None:
            check_full(A, B, C, m, k, n, f"{(m, k, n)} p={p} {name}")
            first = C
        else:
            assert np.array_equal(C, first), f"{(m, k, n)} p={p} {name}: bits differ"


def test_batch_4096_log_uniform(g):
    """4096 products, m, k, n log-uniform in [64, 4096), in one graph-captured persistent launch
    under every policy the benchmark uses.  Under the first policy every row of every product is
    checked with Freivalds' test (64 random vectors, so a dropped or misrouted tile of any product
    fails) and four sampled rows of each product against the oracle; the other policies must give
    the same bits."""
    import torch
    count = 4096
    dims = [tuple(int(x) for x in r) for r in synth.log_uniform_dims(3, 4, count, 64, 4096)]
    print(f"batch of {count}: generating", flush=True)
    host, probs = [], []
    for i, (m, k, n) in enumerate(dims):
        A = synth.uniform(5000 + i, synth.TAG_A, m, k)
        B = synth.uniform(5000 + i, synth.TAG_B, k, n)
        dA, dB = to_dev(A), to_dev(B)
        dC = torch.zeros((m, (n + 63) // 64), dtype=torch.int64, device="cuda")
        host.append((A, B, dA, dB, dC))
        probs.append(g.problem(dC, dA, dB, m, k, n))
    policies = [("fixed", g.POLICY_FIXED)]
    import os
    if os.path.exists(g.DEFAULT_MODEL):
        policies.append(("model", g.POLICY_MODEL))
    first = None
    try:
        for name, pol in policies:
            print(f"batch of {count}: policy {name}", flush=True)
            if pol == g.POLICY_MODEL:
                g.load_model()
            g.set_policy(pol)
            for h in host:
                h[4].zero_()
            g.mul_batched(probs)
            torch.cuda.synchronize()
            outs = [from_dev(h[4]) for h in host]
            if first is None:
                for i, ((m, k, n), (A, B, *_), C) in enumerate(zip(dims, host, outs)):
                    rows = np.unique(np.linspace(0, m - 1, 4).astype(np.int64))
                    assert np.array_equal(C[rows], oracle.mul_rows(A, B, m, k, n, rows)), f"product {(m, k, n)}"
                    X = synth.uniform(9000 + i, TAG_FREIVALDS, n, 64)
                    CX = oracle.mul(C, X, m, n, 64)
                    ABX = oracle.mul(A, oracle.mul(B, X, k, n, 64), m, k, 64)
                    assert np.array_equal(CX, ABX), f"product {i} {(m, k, n)}: Freivalds test failed"
                    if n % 64:
                        assert not np.any(C[:, -1] >> np.uint64(n % 64)), f"product {i}: padding bits of C not zero"
                first = outs
            else:
                for a, b, d in zip(first, outs, dims):
                    assert np.array_equal(a, b), f"policy {name} changed the bits of {d}"
    finally:
        g.set_policy(g.POLICY_FIXED)
        g.set_model(None)


def test_largest_square_65536(g):
    """Twice the headline size: 65536 x 65536 operands (512 MiB each) under the library's own
    schedule (three Strassen-Winograd levels, 343 leaves in several grouped launches), checked
    like the benchmarked sizes."""
    n = 65536
    A = synth.uniform(1, synth.TAG_A, n, n)
    B = synth.uniform(1, synth.TAG_B, n, n)
    s = g.resolve_schedule(n, n, n)
    print(f"n={n} library schedule kernel {s.kernel} variant {s.variant} cutoff {s.cutoff} splitk {s.splitk}",
          flush=True)
    C = run(g, A, B, n, n, n, None, ldc_pad=0)
    check_full(A, B, C, n, n, n, f"{n}^3 library")
