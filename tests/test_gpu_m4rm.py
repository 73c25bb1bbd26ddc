"""GPU parity of the M4RM base case, split-K and Strassen-Winograd against the CPU oracle.

Every comparison is bit-exact: over GF(2) the product is unique.
"""
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


def M4RM(variant=0, cutoff=0, splitk=1, odd=0, kappa=0, memory=0):
    import paper_0811_1714_amd as g
    return g.Schedule(g.KERNEL_M4RM, variant, cutoff, splitk, odd, kappa, memory)


# Tiles that offer tables narrower than 8 bits (Section 3.1's k): every tile of at most 1024 rows.
KAPPA_VARIANTS = (1, 2, 3, 4, 12, 13, 18, 19, 20)


def test_config_1024_square_plain_m4rm(g):
    # 1024 x 1024 times 1024 x 1024, Bernoulli(1/2), M4RM with 8-bit tables, no Strassen.
    for v in range(g.kernel_variants(g.KERNEL_M4RM)):
        print(f"1024^3 variant {v}", flush=True)
        run_and_check(g, 1024, 1024, 1024, schedule=M4RM(v), garbage=False, seed=0)


SHAPES = [(1, 1, 1), (1, 64, 64), (7, 9, 130), (64, 64, 64), (65, 65, 65), (127, 200, 63), (129, 129, 129),
          (300, 777, 129), (1000, 513, 2049), (769, 1025, 2048), (2047, 31, 4097), (33, 5000, 70)]


@pytest.mark.parametrize("m,k,n", SHAPES)
def test_shape_grid_all_variants(g, m, k, n):
    for v in range(g.kernel_variants(g.KERNEL_M4RM)):
        print(f"shape {(m, k, n)} variant {v}", flush=True)
        run_and_check(g, m, k, n, schedule=M4RM(v), seed=m + k + n, lda_pad=1, ldb_pad=3, ldc_pad=2)


@pytest.mark.parametrize("m,k,n", SHAPES)
def test_shape_grid_narrow_tables(g, m, k, n):
    """Every tile with narrow tables at every width 4..7: A's kappa-bit fields become index bytes
    (fields straddling words, a last field cut short by k, garbage padding bits past k)."""
    for v in KAPPA_VARIANTS:
        for kappa in (4, 5, 6, 7):
            print(f"shape {(m, k, n)} variant {v} kappa {kappa}", flush=True)
            run_and_check(g, m, k, n, schedule=M4RM(v, kappa=kappa), seed=m + k + n + kappa, lda_pad=1, ldb_pad=3,
                          ldc_pad=2)


@pytest.mark.parametrize("shape,sched", [
    ((1000, 1000, 1000), (2, 100, 1, 0, 5)),        # two Strassen levels over 5-bit tables
    ((1025, 1023, 1021), (1, 256, 1, 1, 7)),        # peeling: inner-slice and edge fix-ups expanded too
    ((300, 1000, 3000), (3, 0, 4, 0, 6)),           # k in four slices, each expanded on its own
    ((4095, 65537, 129), (13, 0, 1, 0, 4)),         # long k: 16385 index bytes per row
    ((2047, 31, 4097), (19, 0, 1, 0, 5)),           # k shorter than one phase
])
def test_narrow_tables_with_recursion_split_and_peeling(g, shape, sched):
    m, k, n = shape
    v, cutoff, sk, odd, kappa = sched
    print(f"narrow {(m, k, n)} variant {v} cutoff {cutoff} splitk {sk} odd {odd} kappa {kappa}", flush=True)
    base = run_and_check(g, m, k, n, schedule=M4RM(v, cutoff, sk, odd, kappa), seed=21, lda_pad=2, ldc_pad=1)
    wide = run_and_check(g, m, k, n, schedule=M4RM(v, cutoff, sk, odd), seed=21, lda_pad=2, ldc_pad=1)
    assert np.array_equal(base, wide)
    run_and_check(g, m, k, n, schedule=M4RM(v, cutoff, sk, odd, kappa), accumulate=True, seed=22, ldb_pad=1)


@pytest.mark.parametrize("m,k,n,cutoff,variant", [
    (2048, 2048, 2048, 512, 1),      # two-temporary top level, one breadth-first level below
    (1024, 1500, 1024, 256, 3),      # k halves unequal (k1 < k0): S3, T3 and P1..P3 use k1
    (1536, 777, 2560, 300, 18),      # two levels below the top
    (3000, 3000, 3000, 1024, 16),    # four-table leaves
])
def test_two_temporary_schedule_same_bits(g, m, k, n, cutoff, variant):
    """Section 4's memory-efficient schedule (two temporaries at the top level, products written
    straight into C's quadrants) gives the breadth-first schedule's bits."""
    print(f"two-temporary {(m, k, n)} cutoff {cutoff} variant {variant}", flush=True)
    low = run_and_check(g, m, k, n, schedule=M4RM(variant, cutoff, memory=1), seed=31, lda_pad=1, ldb_pad=2,
                        ldc_pad=1)
    fast = run_and_check(g, m, k, n, schedule=M4RM(variant, cutoff), seed=31, lda_pad=1, ldb_pad=2, ldc_pad=1)
    assert np.array_equal(low, fast)


@pytest.mark.parametrize("m,k,n,cutoff,acc", [(1024, 1024, 1024, 256, False), (2048, 1536, 1280, 384, True),
                                               (1024, 2048, 512, 200, False)])
def test_fused_two_level_passes(g, m, k, n, cutoff, acc):
    """Two recursion levels with exact splits (m a multiple of 4, k and n of 256) run both levels'
    pre-additions in one pass and both levels' post-additions in another; the bits must equal the
    oracle's and those of the same product one level deeper and one level shallower."""
    print(f"fused passes {(m, k, n)} cutoff {cutoff} accumulate {acc}", flush=True)
    two = run_and_check(g, m, k, n, schedule=M4RM(1, cutoff), accumulate=acc, seed=33, ldc_pad=1, lda_pad=1)
    one = run_and_check(g, m, k, n, schedule=M4RM(1, 2 * cutoff), accumulate=acc, seed=33, ldc_pad=1, lda_pad=1)
    three = run_and_check(g, m, k, n, schedule=M4RM(1, cutoff // 2), accumulate=acc, seed=33, ldc_pad=1, lda_pad=1)
    assert np.array_equal(two, one) and np.array_equal(two, three)


def test_two_temporary_schedule_falls_back(g):
    """Where the two-temporary form does not apply (odd rows, columns not a multiple of 128,
    accumulation) the call runs breadth-first, with the same bits."""
    for (m, k, n, acc) in [(1025, 1024, 1024, False), (1024, 1024, 1000, False), (1024, 1024, 1024, True)]:
        print(f"two-temporary fallback {(m, k, n)} accumulate {acc}", flush=True)
        run_and_check(g, m, k, n, schedule=M4RM(1, 256, memory=1), accumulate=acc, seed=32)


@pytest.mark.parametrize("m,k,n", [(100, 300, 70), (513, 2048, 2100), (64, 65, 4096)])
def test_addmul_semantics(g, m, k, n):
    print(f"addmul {(m, k, n)}", flush=True)
    run_and_check(g, m, k, n, schedule=M4RM(0), accumulate=True, seed=3, ldc_pad=1)
    run_and_check(g, m, k, n, accumulate=True, seed=4)


@pytest.mark.parametrize("m,k,n,sk", [(100, 4096, 129, 4), (4095, 6553, 129, 32), (300, 1000, 3000, 7)])
def test_split_k(g, m, k, n, sk):
    print(f"split-k {(m, k, n, sk)}", flush=True)
    run_and_check(g, m, k, n, schedule=M4RM(2, 0, sk), seed=5, ldc_pad=1)
    run_and_check(g, m, k, n, schedule=M4RM(2, 0, sk), accumulate=True, seed=6)


@pytest.mark.parametrize("m,k,n", [(1000, 777, 1300), (2049, 100, 70), (513, 4100, 520)])
def test_algorithm1_tile_accumulate_and_split_k(g, m, k, n):
    # Algorithm 1's tile (C updated in global memory once per stripe) in every output mode:
    # store, accumulate, and the atomic XOR of a k split.
    print(f"Algorithm 1 {(m, k, n)}", flush=True)
    run_and_check(g, m, k, n, schedule=M4RM(21), accumulate=True, seed=16, ldc_pad=1)
    run_and_check(g, m, k, n, schedule=M4RM(21, 0, 3), seed=17, lda_pad=1)
    run_and_check(g, m, k, n, schedule=M4RM(21, 0, 5), accumulate=True, seed=18)


@pytest.mark.parametrize("m,k,n,cutoff", [(256, 256, 256, 64), (300, 200, 500, 64), (1000, 1000, 1000, 100),
                                          (777, 1500, 1300, 300), (2049, 2049, 2049, 512), (1025, 130, 1025, 64)])
def test_strassen_winograd_any_cutoff_same_bits(g, m, k, n, cutoff):
    print(f"strassen {(m, k, n)} cutoff {cutoff}", flush=True)
    base = run_and_check(g, m, k, n, schedule=M4RM(0, 0), seed=7)
    got = run_and_check(g, m, k, n, schedule=M4RM(0, cutoff), seed=7)
    assert np.array_equal(base, got)
    run_and_check(g, m, k, n, schedule=M4RM(3, cutoff), seed=8, accumulate=True, ldc_pad=1)


@pytest.mark.parametrize("m,k,n,cutoff", [(257, 257, 257, 64), (1025, 1023, 1021, 256), (300, 777, 129, 64),
                                          (2049, 2050, 2051, 512), (1001, 3000, 700, 128), (130, 4097, 1000, 64)])
def test_peeling_same_bits_as_padding(g, m, k, n, cutoff):
    # Section 4: peeling and (virtual) padding reach the same product.
    print(f"peel {(m, k, n)} cutoff {cutoff}", flush=True)
    pad = run_and_check(g, m, k, n, schedule=M4RM(1, cutoff), seed=12)
    peel = run_and_check(g, m, k, n, schedule=M4RM(1, cutoff, odd=1), seed=12)
    assert np.array_equal(pad, peel)
    run_and_check(g, m, k, n, schedule=M4RM(3, cutoff, odd=1), seed=13, accumulate=True, ldc_pad=1, lda_pad=1)
    run_and_check(g, m, k, n, schedule=M4RM(16, cutoff, odd=1), seed=15, ldb_pad=1)
    import paper_0811_1714_amd as gg
    run_and_check(g, m, k, n, schedule=gg.Schedule(gg.KERNEL_MFMA, 0, cutoff, 1, 1), seed=14, ldb_pad=2)
    run_and_check(g, m, k, n, schedule=gg.Schedule(gg.KERNEL_CUBIC, 0, cutoff, 1, 1), seed=15)


def test_degenerate_shapes(g):
    for (m, k, n) in [(0, 5, 5), (5, 0, 5), (5, 5, 0), (1, 0, 1), (3, 1, 1), (1, 1, 200)]:
        print(f"degenerate {(m, k, n)}", flush=True)
        run_and_check(g, m, k, n, seed=9, ldc_pad=1)
        run_and_check(g, m, k, n, seed=9, accumulate=True)


def test_sparse_inputs(g):
    print("p = 0.01", flush=True)
    run_and_check(g, 1000, 3000, 2000, p=0.01, seed=10)


def test_repeat_runs_identical(g):
    print("repeat", flush=True)
    run_and_check(g, 1500, 1500, 1500, schedule=M4RM(1), seed=11, repeat=3)


def test_wide_strides_use_the_fallback_tiles(g):
    """Rows of 2^20 words or more overflow the 32-bit offsets some tiles use: the four-table
    tiles hand such an A to the 1408-row two-table tile, the one-word tiles hand such a B to
    the eight-table tile.  The bits must not change."""
    for v in (16, 17, 18, 22):
        print(f"lda >= 2^20, variant {v}", flush=True)
        run_and_check(g, 3, 100, 700, schedule=M4RM(v), seed=41, lda_pad=1 << 20)
    for v in (14, 15):
        print(f"ldb >= 2^20, variant {v}", flush=True)
        run_and_check(g, 300, 17, 50, schedule=M4RM(v), seed=42, ldb_pad=1 << 20)
