"""GPU parity of the other base cases (int8 matrix core, popcount) against the CPU oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from gf2_testutil import run_and_check


@pytest.fixture(scope="module")
def g():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0811_1714_amd as g
    g.lib()
    return g


def S(kernel, variant=0, cutoff=0, splitk=1):
    import paper_0811_1714_amd as g
    return g.Schedule(kernel, variant, cutoff, splitk)


MFMA_SHAPES = [(1, 1, 1), (32, 32, 32), (33, 65, 31), (256, 256, 256), (257, 300, 511), (1024, 1024, 1024),
               (100, 4096, 70), (700, 129, 1300)]


@pytest.mark.parametrize("m,k,n", MFMA_SHAPES)
def test_mfma_parity_grid(g, m, k, n):
    print(f"mfma {(m, k, n)}", flush=True)
    run_and_check(g, m, k, n, schedule=S(g.KERNEL_MFMA), seed=m + 2 * k + 3 * n, lda_pad=1, ldb_pad=2, ldc_pad=1)


def test_mfma_addmul_splitk_strassen(g):
    print("mfma addmul / split-k / strassen", flush=True)
    run_and_check(g, 300, 700, 500, schedule=S(g.KERNEL_MFMA), accumulate=True, seed=21, ldc_pad=1)
    run_and_check(g, 200, 5000, 129, schedule=S(g.KERNEL_MFMA, 0, 0, 8), seed=22)
    base = run_and_check(g, 1500, 1300, 1100, schedule=S(g.KERNEL_M4RM), seed=23)
    got = run_and_check(g, 1500, 1300, 1100, schedule=S(g.KERNEL_MFMA, 0, 300), seed=23)
    assert np.array_equal(base, got)


CUBIC_SHAPES = [(1, 1, 1), (5, 64, 64), (17, 65, 1), (64, 130, 129), (333, 1000, 200), (1024, 1024, 1024),
                (4095, 6553, 129), (100, 300, 64)]


@pytest.mark.parametrize("m,k,n", CUBIC_SHAPES)
def test_cubic_popcount_grid(g, m, k, n):
    print(f"cubic {(m, k, n)}", flush=True)
    run_and_check(g, m, k, n, schedule=S(g.KERNEL_CUBIC), seed=m + 5 * k + 7 * n, lda_pad=2, ldb_pad=1, ldc_pad=1)


NARROW_SHAPES = [(1, 1, 1), (3, 64, 2), (1000, 5000, 3), (4097, 129, 8), (300, 70000, 2), (257, 4100, 5),
                 (64, 131072, 1), (2049, 8193, 4)]


@pytest.mark.parametrize("m,k,n", NARROW_SHAPES)
def test_cubic_narrow_streaming(g, m, k, n):
    """At most eight columns of B: the popcount base case streams A against B's columns held in
    LDS.  Ragged k, garbage in every padding, wide strides, both output modes, k slices."""
    print(f"narrow {(m, k, n)}", flush=True)
    run_and_check(g, m, k, n, schedule=S(g.KERNEL_CUBIC), seed=m + 3 * k + 11 * n, lda_pad=3, ldb_pad=2, ldc_pad=1)
    run_and_check(g, m, k, n, schedule=S(g.KERNEL_CUBIC), accumulate=True, seed=m + k + n, ldc_pad=2)
    if k >= 1024:
        run_and_check(g, m, k, n, schedule=S(g.KERNEL_CUBIC, 0, 0, 4), seed=m + 2 * k + n)


def test_mfma_narrow_products_in_one_launch(g):
    """The int8 base keeps every product's B transposed in its own scratch slice; products of at
    most eight columns (k slices, peeling fix-ups) must get slices of the transposed size,
    not of the narrow popcount's."""
    run_and_check(g, 1000, 9000, 3, schedule=S(g.KERNEL_MFMA, 0, 0, 4), seed=61)
    run_and_check(g, 2049, 2050, 2051, schedule=g.Schedule(g.KERNEL_MFMA, 0, 512, 1, 1), seed=62, ldb_pad=2)


def test_cubic_addmul_splitk_strassen(g):
    print("cubic addmul / split-k / strassen", flush=True)
    run_and_check(g, 300, 700, 500, schedule=S(g.KERNEL_CUBIC), accumulate=True, seed=31, ldc_pad=1)
    run_and_check(g, 200, 5000, 129, schedule=S(g.KERNEL_CUBIC, 0, 0, 8), seed=32)
    base = run_and_check(g, 900, 1300, 700, schedule=S(g.KERNEL_M4RM), seed=33)
    got = run_and_check(g, 900, 1300, 700, schedule=S(g.KERNEL_CUBIC, 0, 300), seed=33)
    assert np.array_equal(base, got)
