"""GPU parity of the batched persistent executor: every product of a batch against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

import oracle
import synth
from gf2_testutil import from_dev, operand, to_dev


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    return g


def make_batch(g, dims, seed, schedules=None, accumulate=None, rows_check=None):
    """Device operands and problems; returns (problems, host data needed for checking)."""
    probs, host = [], []
    for i, (m, k, n) in enumerate(dims):
        A = operand(seed + i, synth.TAG_A, m, k, ld=(k + 63) // 64 + (i % 2), garbage=True)
        B = operand(seed + i, synth.TAG_B, k, n, ld=(n + 63) // 64 + (i % 3 == 0), garbage=True)
        C0 = synth.uniform(seed + i, synth.TAG_C, m, n, ld=(n + 63) // 64 + 1)
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C0)
        acc = bool(accumulate[i]) if accumulate is not None else False
        sch = schedules[i] if schedules is not None else -1
        probs.append(g.problem(dC, dA, dB, m, k, n, accumulate=acc, schedule=sch))
        host.append((A, B, C0, dA, dB, dC, acc))
    return probs, host


def check_batch(dims, host, rows_per_product=None):
    for (m, k, n), (A, B, C0, dA, dB, dC, acc) in zip(dims, host):
        got = from_dev(dC)
        W = (n + 63) // 64
        if rows_per_product is None:
            ref = oracle.mul(A, B, m, k, n)
            rows = np.arange(m)
        else:
            rows = np.unique(np.linspace(0, m - 1, min(m, rows_per_product)).astype(np.int64))
            ref = oracle.mul_rows(A, B, m, k, n, rows)
        expect = (C0[rows, :W] ^ ref) if acc else ref
        assert oracle.equal_packed(got[rows, :W], expect, n), f"product {(m, k, n)} differs"
        assert np.all(got[:, W:] == C0[:, W:]), "stride gap written"


def test_mixed_schedules_small_batch(g):
    import torch
    rng = np.random.default_rng(5)
    dims = [tuple(int(x) for x in rng.integers(1, 700, size=3)) for _ in range(48)]
    nc = g.num_candidates()
    schedules = [int(i % (nc + 1)) - 1 for i in range(len(dims))]        # -1 and every candidate
    accumulate = [i % 5 == 0 for i in range(len(dims))]
    print(f"batch of {len(dims)} mixed schedules", flush=True)
    probs, host = make_batch(g, dims, 100, schedules, accumulate)
    g.mul_batched(probs)
    torch.cuda.synchronize()
    check_batch(dims, host)


def test_replay_and_schedule_independence(g):
    import torch
    dims = [(300, 500, 700), (1025, 64, 129), (64, 2000, 64), (2100, 2100, 2100), (1, 1, 1), (700, 0, 80)]
    print("replay", flush=True)
    probs, host = make_batch(g, dims, 200)
    g.mul_batched(probs)
    torch.cuda.synchronize()
    first = [from_dev(h[5]).copy() for h in host]
    for h in host:
        h[5].copy_(to_dev(h[2]))
    g.mul_batched(probs)            # cached graph, counter reset by its own kernel
    torch.cuda.synchronize()
    second = [from_dev(h[5]).copy() for h in host]
    for a, b in zip(first, second):
        assert np.array_equal(a, b)
    check_batch(dims, host)
    for sched in range(g.num_candidates()):
        probs2 = [g.Problem(p.A, p.B, p.C, p.m, p.k, p.n, p.lda, p.ldb, p.ldc, 0, sched) for p in probs]
        for h in host:
            h[5].copy_(to_dev(h[2]))
        g.mul_batched(probs2)
        torch.cuda.synchronize()
        for a, h in zip(first, host):
            assert np.array_equal(a, from_dev(h[5])), f"schedule {sched} changed the bits"


def test_plan_api_and_uneven_batch(g):
    import torch
    dims = [tuple(int(x) for x in row) for row in synth.log_uniform_dims(7, 9, 256, 64, 4096)]
    print("plan api, 256 log-uniform products", flush=True)
    probs, host = make_batch(g, dims, 300)
    plan = g.BatchPlan(probs)
    assert all(0 <= plan.schedule(i) < g.num_candidates() for i in range(len(dims)))
    plan.execute()
    torch.cuda.synchronize()
    check_batch(dims, host, rows_per_product=8)
    plan.destroy()


def test_batch_alias_rejected_and_nothing_written(g):
    import torch
    A = to_dev(synth.uniform(1, 1, 64, 64))
    B = to_dev(synth.uniform(1, 2, 64, 64))
    C = to_dev(np.zeros((64, 1), dtype=np.uint64))
    probs = [g.problem(C, A, B, 64, 64, 64), g.problem(A, C, B, 64, 64, 64)]   # 2nd writes the 1st's A
    with pytest.raises(g.GF2Error) as e:
        g.mul_batched(probs)
    assert e.value.status == 2
    torch.cuda.synchronize()
    assert np.all(from_dev(C) == 0)
