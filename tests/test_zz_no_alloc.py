"""gf2_mul_noalloc: the product computed in the library's static device scratch array instead of
its allocated workspace.  Through the C ABI, each call is compared bit for bit with
gf2_mul_sched on the same inputs and schedule (and with the oracle); two calls in a row, the
second smaller, so the second runs in the array the first left dirty."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
import synth
from gf2_testutil import SENTINEL, from_dev, to_dev


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    g.set_policy(g.POLICY_FIXED)
    return g


def _operands(seed, m, k, n, pad=1):
    A = synth.garbage_padding(synth.uniform(seed, synth.TAG_A, m, k, ld=(k + 63) // 64 + pad), k, seed=seed + 1)
    B = synth.garbage_padding(synth.uniform(seed, synth.TAG_B, k, n, ld=(n + 63) // 64 + pad), n, seed=seed + 2)
    C0 = synth.garbage_padding(synth.uniform(seed, synth.TAG_C, m, n, ld=(n + 63) // 64 + pad), n, seed=seed + 3)
    C0[:, (n + 63) // 64:] = SENTINEL
    return A, B, C0


def _run(g, fn, A, B, C0, m, k, n, sched, accumulate):
    import torch
    dA, dB, dC = to_dev(A), to_dev(B), to_dev(C0)
    fn(dC.data_ptr(), dC.stride(0), dA.data_ptr(), dA.stride(0), dB.data_ptr(), dB.stride(0), m, k, n,
       accumulate=accumulate, schedule=sched)
    torch.cuda.synchronize()
    return from_dev(dC)


CALLS = [
    # (label, m, k, n, kernel, variant, cutoff, accumulate): each pair runs in order, the second smaller
    ("strassen one level then a smaller two-level product", [
        (2304, 2100, 2500, 1, 1, 1024, False),
        (1500, 1300, 1700, 1, 3, 384, False),
    ]),
    ("accumulate, one level then a smaller two-level product", [
        (2100, 2300, 1900, 1, 2, 1024, True),
        (700, 900, 650, 1, 4, 256, True),
    ]),
    ("popcount and int8 matrix-core base cases (scratch holds B transposed)", [
        (1000, 3000, 700, 3, 0, 0, False),
        (600, 2000, 500, 2, 0, 0, False),
    ]),
]


@pytest.mark.parametrize("label,calls", CALLS, ids=[c[0] for c in CALLS])
def test_noalloc_matches_allocating_entry_point(g, label, calls):
    for i, (m, k, n, kern, var, cut, acc) in enumerate(calls):
        print(f"noalloc: {label} call {i}: {(m, k, n)} kernel {kern} variant {var} cutoff {cut} acc {acc}", flush=True)
        s = g.Schedule(kern, var, cut, 1)
        need = g.workspace_bytes(m, k, n, s)
        assert 0 < need <= g.NOALLOC_SCRATCH_BYTES, "the case must use the scratch array"
        A, B, C0 = _operands(40 + i, m, k, n)
        got = _run(g, g.mul_noalloc_ptr, A, B, C0, m, k, n, s, acc)
        ref = _run(g, g.mul_ptr, A, B, C0, m, k, n, s, acc)
        assert np.array_equal(got, ref), "gf2_mul_noalloc differs from gf2_mul_sched"
        W = (n + 63) // 64
        prod = oracle.mul(A, B, m, k, n)
        expect = (C0[:, :W] ^ prod) if acc else prod
        assert oracle.equal_packed(got[:, :W], expect, n), "gf2_mul_noalloc differs from the oracle"
        assert np.all(got[:, W:] == SENTINEL), "stride-gap words of C were written"


def test_noalloc_library_choice_and_too_large(g):
    import torch
    # The library's own schedule (sched NULL) for a product whose default needs no workspace.
    m, k, n = 1024, 1024, 1024
    A, B, C0 = _operands(7, m, k, n)
    got = _run(g, g.mul_noalloc_ptr, A, B, C0, m, k, n, None, False)
    assert oracle.equal_packed(got[:, :16], oracle.mul(A, B, m, k, n), n)
    # Two Strassen levels at 8192^3 need more than the array holds: rejected, C untouched.
    m = k = n = 8192
    s = g.Schedule(g.KERNEL_M4RM, 16, 2048, 1)
    assert g.workspace_bytes(m, k, n, s) > g.NOALLOC_SCRATCH_BYTES
    dA = torch.zeros((m, 128), dtype=torch.int64, device="cuda")
    dB = torch.zeros((k, 128), dtype=torch.int64, device="cuda")
    dC = torch.full((m, 128), 5, dtype=torch.int64, device="cuda")
    with pytest.raises(g.GF2Error) as e:
        g.mul_noalloc_ptr(dC.data_ptr(), 128, dA.data_ptr(), 128, dB.data_ptr(), 128, m, k, n, schedule=s)
    assert e.value.status == 6 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((dC == 5).all()), "a rejected call wrote C"
