"""Helpers shared by the GPU tests: seeded operands, device transfer, oracle comparison."""
import numpy as np

import oracle
import synth


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def from_dev(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def operand(seed, tag, rows, cols, ld=None, garbage=False, p=0.5):
    a = synth.bernoulli(seed, tag, rows, cols, p, ld=ld)
    return synth.garbage_padding(a, cols, seed=seed * 7 + tag) if garbage else a


SENTINEL = np.uint64(0xA5A5A5A5DEADBEEF)


def run_and_check(g, m, k, n, *, schedule=None, accumulate=False, seed=1, lda_pad=0, ldb_pad=0, ldc_pad=0,
                  garbage=True, p=0.5, repeat=1):
    """Run one product on the GPU and compare every valid bit with the oracle; also check that
    stride-gap words of C are untouched and (mul) that C's padding bits are zero."""
    import torch
    Wk, Wn = (k + 63) // 64, (n + 63) // 64
    A = operand(seed, synth.TAG_A, m, k, ld=max(Wk, 1) + lda_pad, garbage=garbage, p=p)
    B = operand(seed, synth.TAG_B, k, n, ld=max(Wn, 1) + ldb_pad, garbage=garbage, p=p)
    ldc = max(Wn, 1) + ldc_pad
    C0 = synth.garbage_padding(synth.uniform(seed, synth.TAG_C, m, n, ld=ldc), n, seed=seed + 5)
    if ldc > Wn:
        C0[:, Wn:] = SENTINEL
    ref = oracle.mul(A, B, m, k, n)
    dA, dB = to_dev(A), to_dev(B)
    outs = []
    for _ in range(repeat):
        dC = to_dev(C0)
        g.mul(dC, dA, dB, m, k, n, accumulate=accumulate, schedule=schedule)
        torch.cuda.synchronize()
        outs.append(from_dev(dC))
    for C in outs:
        if accumulate:
            expect = C0[:, :Wn] ^ ref
            assert oracle.equal_packed(C[:, :Wn], expect, n), "addmul result differs from the oracle"
            if Wn and n % 64:
                keep = ~np.uint64((1 << (n % 64)) - 1)
                assert np.array_equal(C[:, Wn - 1] & keep, C0[:, Wn - 1] & keep), "addmul touched padding bits"
        else:
            assert oracle.equal_packed(C[:, :Wn], ref, n), "product differs from the oracle"
            assert np.array_equal(C[:, :Wn], ref), "padding bits of C not written as zero"
        if ldc > Wn:
            assert np.all(C[:, Wn:] == SENTINEL), "stride-gap words of C were written"
    for C in outs[1:]:
        assert np.array_equal(C, outs[0]), "repeated runs differ"
    return outs[0]
