"""Single products under HIP graph capture: once the workspace is reserved, gf2_mul enqueues
kernels only (no allocation, no host synchronisation, no memset nodes), so a caller may
capture it.  Each graph is replayed several times with eager work in between, and every
replay is checked against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
import synth
from gf2_testutil import from_dev, to_dev


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    return g


CASES = [
    ("strassen two levels, 1408-row tiles, k-split tail", 8192, 4096, 8192, (4, 2048, 1)),
    ("k split into 8 slices", 3000, 9000, 1000, (2, 0, 8)),
    ("odd sizes, peeling", 2049, 2050, 2051, (1, 512, 1, 1)),
    ("matrix-vector, one-word tiles", 20000, 20000, 1, (14, 0, 8)),
    ("four-table tiles, one level", 8192, 8192, 4100, (16, 4096, 1)),
]


@pytest.mark.parametrize("name,m,k,n,sched", CASES, ids=[c[0] for c in CASES])
def test_captured_product_replays(g, name, m, k, n, sched):
    import torch
    print(f"graph: {name} {(m, k, n)}", flush=True)
    A = synth.uniform(31, synth.TAG_A, m, k)
    B = synth.uniform(31, synth.TAG_B, k, n)
    rows = np.unique(np.linspace(0, m - 1, 48).astype(np.int64))
    ref = oracle.mul_rows(A, B, m, k, n, rows)
    dA, dB = to_dev(A), to_dev(B)
    W = (n + 63) // 64
    dC = torch.zeros((m, W), dtype=torch.int64, device="cuda")
    s = g.Schedule(g.KERNEL_M4RM, *sched)
    g.set_policy(g.POLICY_FIXED)
    g.reserve_workspace(g.workspace_bytes(m, k, n, s))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.mul(dC, dA, dB, m, k, n, schedule=s, stream=side)      # warm-up outside capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        g.mul(dC, dA, dB, m, k, n, schedule=s, stream=side)
    for rep in range(3):
        dC.fill_(-1)                                               # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = from_dev(dC)
        assert np.array_equal(got[rows, :W], ref), f"replay {rep} differs from the oracle"
        if n % 64:
            assert not np.any(got[:, W - 1] >> np.uint64(n % 64)), "padding bits not zero"
    del graph


def test_captured_workspace_survives_a_larger_eager_product(g):
    """A graph captured on a Strassen-Winograd product keeps the workspace address it was
    captured with.  A later, larger eager product must not free that buffer (it grows into a
    new one), so replays after it still give the oracle's bits."""
    import torch
    m = k = n = 2048
    s = g.Schedule(g.KERNEL_M4RM, 2, 1024, 1)
    A = synth.uniform(41, synth.TAG_A, m, k)
    B = synth.uniform(41, synth.TAG_B, k, n)
    ref = oracle.mul(A, B, m, k, n)
    dA, dB = to_dev(A), to_dev(B)
    dC = torch.zeros((m, n // 64), dtype=torch.int64, device="cuda")
    g.set_policy(g.POLICY_FIXED)
    torch.cuda.synchronize()
    g.shutdown()                       # start from no workspace, so the eager product below must grow it
    g.reserve_workspace(g.workspace_bytes(m, k, n, s))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.mul(dC, dA, dB, m, k, n, schedule=s, stream=side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        g.mul(dC, dA, dB, m, k, n, schedule=s, stream=side)
    # A larger eager product whose workspace exceeds the reserved one.
    M = 8192
    big = g.Schedule(g.KERNEL_M4RM, 2, 2048, 1)
    assert g.workspace_bytes(M, M, M, big) > 4 * g.workspace_bytes(m, k, n, s)
    A2 = synth.uniform(42, synth.TAG_A, M, M)
    B2 = synth.uniform(42, synth.TAG_B, M, M)
    dA2, dB2 = to_dev(A2), to_dev(B2)
    dC2 = torch.zeros((M, M // 64), dtype=torch.int64, device="cuda")
    for rep in range(3):
        g.mul(dC2, dA2, dB2, M, M, M, schedule=big)   # eager; first pass grows the workspace
        dC.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(from_dev(dC), ref), f"replay {rep} after a larger eager product differs"
    rows = np.unique(np.linspace(0, M - 1, 32).astype(np.int64))
    assert np.array_equal(from_dev(dC2)[rows], oracle.mul_rows(A2, B2, M, M, M, rows)), "eager product differs"
    del graph
