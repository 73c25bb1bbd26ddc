"""Failure handling on the GPU, every condition forced from the host (no kernel faults, traps or
hangs): an injected allocation failure (GF2_FAULT_ALLOC=1) and a product that would need new
workspace while its stream is being captured.  Each must return its documented status, leave C
untouched, and leave the library usable for the next call."""
import os

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


def operands(m, k, n, seed):
    A = synth.uniform(seed, synth.TAG_A, m, k)
    B = synth.uniform(seed, synth.TAG_B, k, n)
    return A, B, oracle.mul(A, B, m, k, n)


def test_injected_allocation_failure(g):
    import torch
    m = k = n = 2048
    A, B, ref = operands(m, k, n, 51)
    dA, dB = to_dev(A), to_dev(B)
    s = g.Schedule(g.KERNEL_M4RM, 2, 1024, 1)
    torch.cuda.synchronize()
    g.shutdown()                                     # no workspace: the product must allocate
    dC = torch.full((m, n // 64), -1, dtype=torch.int64, device="cuda")
    os.environ["GF2_FAULT_ALLOC"] = "1"
    try:
        print("fault alloc: single product", flush=True)
        with pytest.raises(g.GF2Error) as ei:
            g.mul(dC, dA, dB, m, k, n, schedule=s)
        assert ei.value.status == 3 and "injected" in str(ei.value)
        torch.cuda.synchronize()
        assert np.all(from_dev(dC) == np.uint64(0xFFFFFFFFFFFFFFFF)), "C written by a refused call"
        print("fault alloc: batch plan", flush=True)
        strassen = [c for c in range(g.num_candidates()) if g.candidate(c).cutoff > 0]
        assert strassen, "no Strassen-Winograd candidate to plan"
        with pytest.raises(g.GF2Error) as ei:
            g.mul_batched([g.problem(dC, dA, dB, m, k, n, schedule=strassen[0])])
        assert ei.value.status == 3
    finally:
        del os.environ["GF2_FAULT_ALLOC"]
    print("fault alloc: recovered", flush=True)
    g.mul(dC, dA, dB, m, k, n, schedule=s)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(dC), ref)


def test_capture_without_reserved_workspace_is_refused(g):
    import torch
    m = k = n = 2048
    A, B, ref = operands(m, k, n, 52)
    dA, dB = to_dev(A), to_dev(B)
    s = g.Schedule(g.KERNEL_M4RM, 2, 1024, 1)
    dC = torch.full((m, n // 64), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g.shutdown()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    status = None
    print("capture without workspace", flush=True)
    with torch.cuda.graph(graph, stream=side):
        try:
            g.mul(dC, dA, dB, m, k, n, schedule=s, stream=side)
        except g.GF2Error as e:
            status = e.status
        dC.add_(0)            # keep the captured graph non-empty
    assert status == 4, "a product needing new workspace under capture must return GF2_ERR_CAPTURE"
    graph.replay()
    torch.cuda.synchronize()
    assert np.all(from_dev(dC) == np.uint64(0xFFFFFFFFFFFFFFFF)), "C written by a refused call"
    del graph
    g.mul(dC, dA, dB, m, k, n, schedule=s)
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(dC), ref)
