"""Pins for the CPU oracle (runs without a GPU).

The oracle is checked against things other than itself: brute force on tiny
inputs, exhaustive small cases including the worked example of Section 3, the
library routine numpy matmul on integers (the product mod 2), algebraic
identities, Freivalds' check, and values printed in the paper.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def rand_bits(rng, r, c, p=0.5):
    return (rng.random((r, c)) < p).astype(np.uint8)


def np_product_bits(Ab, Bb):
    """Library routine: the integer matrix product, reduced mod 2."""
    return ((Ab.astype(np.int64) @ Bb.astype(np.int64)) & 1).astype(np.uint8)


def packed_mul_bits(Ab, Bb, nthreads=0):
    m, k = Ab.shape
    _, n = Bb.shape
    C = oracle.mul(oracle.pack(Ab), oracle.pack(Bb), m, k, n, nthreads=nthreads)
    return oracle.unpack(C, n)


# --------------------------------------------------------------------------- layout

@pytest.mark.parametrize("cols", [1, 7, 63, 64, 65, 130, 200])
def test_pack_matches_numpy_packbits_little_endian(cols):
    rng = np.random.default_rng(cols)
    bits = rand_bits(rng, 5, cols)
    W = (cols + 63) // 64
    padded = np.zeros((5, W * 64), dtype=np.uint8)
    padded[:, :cols] = bits
    ref = np.packbits(padded, axis=1, bitorder="little").view("<u8")
    assert np.array_equal(oracle.pack(bits), ref)
    assert np.array_equal(oracle.unpack(ref, cols), bits)


def test_synth_padding_is_zero_and_garbage_helper_only_touches_padding():
    A = synth.uniform(3, synth.TAG_A, 17, 70, ld=4)
    assert np.all(A[:, 1] >> np.uint64(6) == 0)
    assert np.all(A[:, 2:] == 0)
    G = synth.garbage_padding(A, 70)
    assert oracle.equal_packed(A, G, 70)
    assert not np.array_equal(A, G)


@pytest.mark.parametrize("cols", [1, 5, 63, 64, 65, 127, 130, 191])
def test_equal_packed_sees_every_valid_bit_and_nothing_else(cols):
    """The comparator the GPU checks use: a flip of any valid bit, in any row, makes two packed
    matrices unequal (both argument orders); a flip of a padding bit or of a stride-gap word
    leaves them equal; a different row count is unequal.  Bits are set by position through
    pack(), which is itself pinned against numpy.packbits above."""
    rng = np.random.default_rng(cols)
    rows = 4
    W = (cols + 63) // 64
    ld = W + 2
    X = np.zeros((rows, ld), dtype=np.uint64)
    X[:, :W] = oracle.pack(rand_bits(rng, rows, cols))
    X[:, W:] = rng.integers(0, 1 << 63, size=(rows, ld - W), dtype=np.uint64)
    assert oracle.equal_packed(X, X.copy(), cols)
    for r in range(rows):
        for j in range(cols):
            one = np.zeros((1, cols), dtype=np.uint8)
            one[0, j] = 1
            Z = X.copy()
            Z[r, :W] ^= oracle.pack(one)[0]
            assert not oracle.equal_packed(X, Z, cols), f"flip of valid bit ({r}, {j}) not seen"
            assert not oracle.equal_packed(Z, X, cols), f"flip of valid bit ({r}, {j}) not seen"
        for j in range(cols, 64 * W):
            Z = X.copy()
            Z[r, j >> 6] ^= np.uint64(1) << np.uint64(j & 63)
            assert oracle.equal_packed(X, Z, cols), f"padding bit ({r}, {j}) compared"
        for w in range(W, ld):
            Z = X.copy()
            Z[r, w] = ~Z[r, w]
            assert oracle.equal_packed(X, Z, cols), f"stride-gap word ({r}, {w}) compared"
    assert not oracle.equal_packed(X, X[:-1], cols)
    assert not oracle.equal_packed(X[:-1], X, cols)


def test_splitmix64_published_first_output():
    # splitmix64 seeded with 0: first output 0xE220A8397B1DCDAF (Vigna's reference generator).
    assert synth.splitmix64(0) == 0xE220A8397B1DCDAF


# --------------------------------------------------------------------------- definition

def test_bruteforce_against_pure_python_loops():
    rng = np.random.default_rng(0)
    for (m, k, n) in [(1, 1, 1), (2, 3, 4), (5, 4, 3), (3, 7, 2)]:
        A, B = rand_bits(rng, m, k), rand_bits(rng, k, n)
        C = [[0] * n for _ in range(m)]
        for i in range(m):
            for j in range(n):
                s = 0
                for t in range(k):
                    s ^= int(A[i, t]) & int(B[t, j])
                C[i][j] = s
        assert np.array_equal(oracle.bruteforce(A, B), np.array(C, dtype=np.uint8))


def test_worked_example_of_section_3_all_2x2_pairs():
    # Section 3, k = 1 example: C = A0 B0 + A1 B1 =
    #   [[a0 b0 + a1 b2, a0 b1 + a1 b3], [a2 b0 + a3 b2, a2 b1 + a3 b3]]  (entries a0..a3 row-major).
    for a in itertools.product((0, 1), repeat=4):
        for b in itertools.product((0, 1), repeat=4):
            a0, a1, a2, a3 = a
            b0, b1, b2, b3 = b
            expect = np.array([[(a0 & b0) ^ (a1 & b2), (a0 & b1) ^ (a1 & b3)],
                               [(a2 & b0) ^ (a3 & b2), (a2 & b1) ^ (a3 & b3)]], dtype=np.uint8)
            A = np.array(a, dtype=np.uint8).reshape(2, 2)
            B = np.array(b, dtype=np.uint8).reshape(2, 2)
            assert np.array_equal(packed_mul_bits(A, B), expect)


def test_exhaustive_3x3_against_integer_matmul():
    allm = np.array(list(itertools.product((0, 1), repeat=9)), dtype=np.uint8).reshape(512, 3, 3)
    tallA = allm.reshape(512 * 3, 3)           # every A stacked vertically
    for j in range(0, 512, 7):
        B = allm[j]
        got = packed_mul_bits(tallA, B).reshape(512, 3, 3)
        ref = np.einsum("aik,kj->aij", allm.astype(np.int64), B.astype(np.int64)) & 1
        assert np.array_equal(got, ref.astype(np.uint8))


SIZES = [0, 1, 2, 3, 7, 63, 64, 65, 127, 128, 129, 200]


@pytest.mark.parametrize("m,k,n", [(m, k, n) for m in (1, 3, 65, 129) for k in SIZES for n in (1, 63, 64, 65, 200)])
def test_mul_matches_integer_matmul_grid(m, k, n):
    rng = np.random.default_rng(m * 1000003 + k * 1009 + n)
    A, B = rand_bits(rng, m, k), rand_bits(rng, k, n)
    assert np.array_equal(packed_mul_bits(A, B), np_product_bits(A, B))


def test_mul_matches_bruteforce_and_numpy_up_to_1024():
    rng = np.random.default_rng(7)
    for (m, k, n) in [(1024, 1024, 1024), (300, 777, 129), (64, 1000, 65)]:
        A, B = rand_bits(rng, m, k), rand_bits(rng, k, n)
        got = packed_mul_bits(A, B)
        assert np.array_equal(got, np_product_bits(A, B))
        if m * k * n <= 5e6:
            assert np.array_equal(got, oracle.bruteforce(A, B))


def test_threads_do_not_change_result():
    A = synth.uniform(1, 1, 333, 500)
    B = synth.uniform(1, 2, 500, 300)
    C1 = oracle.mul(A, B, 333, 500, 300, nthreads=1)
    C8 = oracle.mul(A, B, 333, 500, 300, nthreads=8)
    assert np.array_equal(C1, C8)


def test_mul_rows_equals_full_rows():
    A = synth.uniform(5, 1, 400, 333)
    B = synth.uniform(5, 2, 333, 250)
    C = oracle.mul(A, B, 400, 333, 250)
    rows = np.array([0, 5, 399, 200, 5])
    assert np.array_equal(oracle.mul_rows(A, B, 400, 333, 250, rows), C[rows])


# --------------------------------------------------------------------------- identities

def ident(n):
    return oracle.pack(np.eye(n, dtype=np.uint8))


def test_identities():
    m, k, n, p = 70, 130, 65, 90
    A = synth.uniform(2, 1, m, k)
    B = synth.uniform(2, 2, k, n)
    D = synth.uniform(2, 3, n, p)
    E = synth.uniform(2, 4, k, n)
    assert np.array_equal(oracle.mul(ident(m), A, m, m, k), A)               # I*A = A
    assert np.array_equal(oracle.mul(A, ident(k), m, k, k), A)               # A*I = A
    Z = np.zeros_like(A)
    assert np.all(oracle.mul(Z, B, m, k, n) == 0)                            # 0*B = 0
    AB = oracle.mul(A, B, m, k, n)
    assert np.array_equal(oracle.mul(AB, D, m, n, p), oracle.mul(A, oracle.mul(B, D, k, n, p), m, k, p))
    assert np.array_equal(oracle.mul(A, B ^ E, m, k, n), AB ^ oracle.mul(A, E, m, k, n))
    # (AB)^T = B^T A^T
    ABt = oracle.pack(oracle.unpack(AB, n).T)
    BtAt = oracle.mul(oracle.pack(oracle.unpack(B, n).T), oracle.pack(oracle.unpack(A, k).T), n, k, m)
    assert np.array_equal(ABt, BtAt)
    # accumulate: C ^= A*B  equals  C xor (A*B)
    C0 = synth.uniform(2, 5, m, n)
    Cacc = oracle.mul(A, B, m, k, n, C=C0.copy(), accumulate=True)
    assert np.array_equal(Cacc, C0 ^ AB)


def test_freivalds_64_vectors_detects_single_bit_flip():
    m, k, n = 257, 300, 190
    A = synth.uniform(4, 1, m, k)
    B = synth.uniform(4, 2, k, n)
    X = synth.uniform(4, synth.TAG_X, n, 64)
    C = oracle.mul(A, B, m, k, n)
    lhs = oracle.mul(C, X, m, n, 64)
    rhs = oracle.mul(A, oracle.mul(B, X, k, n, 64), m, k, 64)
    assert np.array_equal(lhs, rhs)
    Cbad = C.copy()
    Cbad[100, 1] ^= np.uint64(1 << 17)
    assert not np.array_equal(oracle.mul(Cbad, X, m, n, 64), rhs)


def test_padding_garbage_ignored_and_stride_gaps_untouched():
    m, k, n = 40, 100, 70
    A = synth.garbage_padding(synth.uniform(6, 1, m, k, ld=3), k, seed=1)
    B = synth.garbage_padding(synth.uniform(6, 2, k, n, ld=4), n, seed=2)
    Aclean = synth.uniform(6, 1, m, k)
    Bclean = synth.uniform(6, 2, k, n)
    ref = oracle.mul(Aclean, Bclean, m, k, n)
    sentinel = np.uint64(0xDEADBEEFCAFEF00D)
    C = np.full((m, 5), sentinel, dtype=np.uint64)
    oracle.mul(A, B, m, k, n, C=C)
    assert np.array_equal(C[:, :2], ref)                                      # padding bits written 0
    assert np.all(C[:, 2:] == sentinel)                                       # gap words untouched
    C2 = np.full((m, 5), sentinel, dtype=np.uint64)
    oracle.mul(A, B, m, k, n, C=C2, accumulate=True)
    assert np.array_equal(C2[:, :2] ^ np.full((m, 2), sentinel, dtype=np.uint64), ref)  # padding unchanged


def test_empty_shapes():
    A = np.zeros((0, 1), dtype=np.uint64)
    assert oracle.mul(A, np.zeros((5, 1), dtype=np.uint64), 0, 5, 5).shape == (0, 1)
    # k = 0: the product is the zero matrix
    C = oracle.mul(np.zeros((3, 0), dtype=np.uint64), np.zeros((0, 1), dtype=np.uint64), 3, 0, 10,
                   C=np.full((3, 1), 5, dtype=np.uint64))
    assert np.all(C == 0)


def test_matvec_is_product_with_one_column():
    m, k = 150, 200
    A = synth.uniform(8, 1, m, k)
    v = synth.uniform(8, 2, 1, k)[0]
    y = oracle.matvec(A, v, m, k)
    Bcol = oracle.pack(oracle.unpack(v[None, :], k).T)        # k x 1
    ref = oracle.unpack(oracle.mul(A, Bcol, m, k, 1), 1)[:, 0]
    assert np.array_equal(oracle.unpack(y[None, :], m)[0], ref)


# --------------------------------------------------------------------------- Section 3

def read_golden_gray():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "gray_codes.txt")
    out, cur = {}, None
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("bits"):
            cur = int(line.split()[1])
            out[cur] = []
        else:
            out[cur].append([int(c) for c in line])
    return out


def test_gray_codes_match_figure():
    for bits, codes in read_golden_gray().items():
        assert oracle.gray_code(bits) == codes


def test_gray_code_is_binary_reflected_closed_form():
    # The reflect-and-prefix construction equals g(i) = i xor (i >> 1), and consecutive entries
    # differ in exactly one bit.
    for kb in range(1, 13):
        vals = [oracle._value(c) for c in oracle.gray_code(kb)]
        assert vals == [i ^ (i >> 1) for i in range(1 << kb)]
        assert all(bin(a ^ b).count("1") == 1 for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("kbits", [1, 2, 3, 5, 8])
def test_make_table_entries_and_row_addition_count(kbits):
    rng = np.random.default_rng(kbits)
    Bb = rand_bits(rng, 12, 90)
    Bp = oracle.pack(Bb)
    cnt = [0]
    r = 2
    T = oracle.make_table(Bp, r, kbits, counter=cnt)
    assert cnt[0] == (1 << kbits) - 1          # Section 3.1: 2^k - 1 row additions
    for x in range(1 << kbits):
        expect = np.zeros(Bp.shape[1], dtype=np.uint64)
        for p in range(kbits):                  # bit p from the most significant selects row r+p
            if (x >> (kbits - 1 - p)) & 1 and r + p < 12:
                expect ^= Bp[r + p]
        assert np.array_equal(T[x], expect)


@pytest.mark.parametrize("m,l,n,kbits,tables,block", [
    (20, 16, 70, 4, 1, None), (33, 37, 65, 3, 1, None), (40, 50, 130, 4, 2, None),
    (17, 64, 64, 2, 8, 5), (9, 10, 3, 4, 2, 4), (30, 5, 200, 8, 1, 7)])
def test_m4rm_algorithms_equal_definition(m, l, n, kbits, tables, block):
    rng = np.random.default_rng(m + l + n)
    A, B = rand_bits(rng, m, l), rand_bits(rng, l, n)
    got = oracle.m4rm(A, oracle.pack(B), kbits, tables=tables, block_rows=block)
    assert np.array_equal(oracle.unpack(got, n), np_product_bits(A, B))


# --------------------------------------------------------------------------- Section 4

@pytest.mark.parametrize("m,l,n,cut,odd", [
    (8, 8, 8, 1, "pad"), (16, 16, 16, 2, "pad"), (13, 17, 9, 2, "pad"), (13, 17, 9, 2, "peel"),
    (32, 12, 20, 3, "peel"), (31, 33, 35, 4, "pad")])
def test_strassen_winograd_over_integers_is_the_product(m, l, n, cut, odd):
    # With real subtraction the formulas of Algorithm 4 must give the exact integer product:
    # a wrong sign, operand or index in any of the 15 additions or 7 products fails here.
    rng = np.random.default_rng(m * l * n)
    A = rng.integers(-5, 6, size=(m, l)).astype(np.int64)
    B = rng.integers(-5, 6, size=(l, n)).astype(np.int64)
    got = oracle.strassen_winograd(A, B, oracle.int_ring(), cut, odd=odd)
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("m,l,n,cut,odd", [(64, 64, 64, 8, "pad"), (50, 70, 90, 8, "pad"), (50, 70, 90, 8, "peel")])
def test_strassen_winograd_over_gf2_is_the_product(m, l, n, cut, odd):
    rng = np.random.default_rng(1)
    A, B = rand_bits(rng, m, l), rand_bits(rng, l, n)
    got = oracle.strassen_winograd(A, B, oracle.gf2_ring(), cut, odd=odd)
    assert np.array_equal(got, packed_mul_bits(A, B))


def test_strassen_counts_seven_products_fifteen_additions():
    cnt = {}
    A = np.ones((16, 16), dtype=np.int64)
    oracle.strassen_winograd(A, A, oracle.int_ring(), 2, counter=cnt)
    # 16 -> 8 -> 4 -> 2: nodes = 1 + 7 + 49, leaves = 343
    assert cnt["nodes"] == 57 and cnt["products"] == 7 * 57 and cnt["adds"] == 15 * 57
    assert cnt["base"] == 343


# --------------------------------------------------------------------------- Section 5

def test_paper_tuning_values():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_tuning.txt")
    for line in open(path):
        line = line.split("#")[0].split()
        if not line or line[0] == "machine":
            continue
        _, l2, l1, cs, bs, k, tb = line
        got = oracle.paper_tuning(int(l2), int(l1))
        assert got[:3] == (int(cs), int(bs), int(k))
        if tb != "-":
            assert got[3] == int(tb)
