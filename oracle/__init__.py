"""CPU oracle for GF(2) matrix multiplication -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never imports it, and it never imports
the product (no shared code, headers, tables or constants).  Inputs come from
the separate ``synth`` generator module.

Contents, each a plain statement of what the paper defines:

* ``mul`` / ``mul_rows`` / ``bruteforce`` / ``matvec`` -- the product itself,
  by definition (Sections 1 and 2.3), via the C routines in ``gf2ref.c``.
* ``gray_code`` / ``make_table`` / ``m4rm`` -- the Method of the Four Russians
  (Section 3, Algorithms 1-3) taken step by step, for small inputs.
* ``strassen_winograd`` -- Algorithm 4 over any ring given by add/sub, with
  the crossover of Section 5 and the padding/peeling of Section 4.
* ``paper_tuning`` -- the tuning rule of Section 5.
* ``mlp`` (submodule) -- float64 reference of the schedule model.

Parity: every function here is pinned by ``tests/test_oracle*.py`` against
brute force, the library routine numpy ``matmul`` on integers, identities,
Freivalds' check or values printed in the paper.  Nothing is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def use_library(path: str | None) -> None:
    """Load the C routines from another build of ``gf2ref.c`` (for instance the ``-march=native``
    build the benchmark makes on its own host); None returns to the in-tree build."""
    global _LIB, _PATH
    _PATH = path
    _LIB = None


_PATH = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _PATH or os.path.join(_HERE, "liboracle_gf2.so")
        if not os.path.exists(path):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.gf2ref_mul.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, ctypes.c_int, ctypes.c_int]
        lib.gf2ref_mul.restype = ctypes.c_int
        lib.gf2ref_mul_rows.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, P, I64, ctypes.c_int]
        lib.gf2ref_mul_rows.restype = ctypes.c_int
        lib.gf2ref_mul_bruteforce.argtypes = [P, P, P, I64, I64, I64]
        lib.gf2ref_mul_bruteforce.restype = ctypes.c_int
        lib.gf2ref_matvec.argtypes = [P, P, I64, P, I64, I64]
        lib.gf2ref_matvec.restype = ctypes.c_int
        lib.gf2ref_max_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def max_threads() -> int:
    return int(_lib().gf2ref_max_threads())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def words(cols: int) -> int:
    return (int(cols) + 63) // 64


# ---------------------------------------------------------------------------
# The product by definition (Sections 1, 2.1-2.3)
# ---------------------------------------------------------------------------

def mul(A: np.ndarray, B: np.ndarray, m: int, k: int, n: int, C: np.ndarray | None = None,
        accumulate: bool = False, nthreads: int = 0) -> np.ndarray:
    """C = A*B (or C ^= A*B) on packed uint64 row-major matrices with their own ld."""
    A = np.ascontiguousarray(A, dtype=np.uint64)
    B = np.ascontiguousarray(B, dtype=np.uint64)
    if C is None:
        C = np.zeros((m, words(n)), dtype=np.uint64)
    assert C.dtype == np.uint64 and C.flags.c_contiguous
    lda = A.shape[1] if A.ndim == 2 and A.shape[0] else words(k)
    ldb = B.shape[1] if B.ndim == 2 and B.shape[0] else words(n)
    ldc = C.shape[1] if C.shape[0] else words(n)
    rc = _lib().gf2ref_mul(_ptr(C), ldc, _ptr(A), lda, _ptr(B), ldb, m, k, n, int(accumulate), nthreads)
    if rc != 0:
        raise ValueError(f"gf2ref_mul failed ({rc})")
    return C


def mul_rows(A: np.ndarray, B: np.ndarray, m: int, k: int, n: int, rows, nthreads: int = 0) -> np.ndarray:
    """Rows ``rows`` of A*B, as a (len(rows), ceil(n/64)) packed array."""
    A = np.ascontiguousarray(A, dtype=np.uint64)
    B = np.ascontiguousarray(B, dtype=np.uint64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros((rows.size, words(n)), dtype=np.uint64)
    lda = A.shape[1] if A.shape[0] else words(k)
    ldb = B.shape[1] if B.shape[0] else words(n)
    rc = _lib().gf2ref_mul_rows(_ptr(out), max(words(n), 1), _ptr(A), lda, _ptr(B), ldb, m, k, n,
                                _ptr(rows), rows.size, nthreads)
    if rc != 0:
        raise ValueError(f"gf2ref_mul_rows failed ({rc})")
    return out


def bruteforce(Abits: np.ndarray, Bbits: np.ndarray) -> np.ndarray:
    """Element-wise definition on unpacked 0/1 matrices."""
    Abits = np.ascontiguousarray(Abits, dtype=np.uint8)
    Bbits = np.ascontiguousarray(Bbits, dtype=np.uint8)
    m, k = Abits.shape
    k2, n = Bbits.shape
    assert k == k2
    C = np.zeros((m, n), dtype=np.uint8)
    _lib().gf2ref_mul_bruteforce(_ptr(C), _ptr(Abits), _ptr(Bbits), m, k, n)
    return C


def matvec(A: np.ndarray, v: np.ndarray, m: int, k: int) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.uint64)
    v = np.ascontiguousarray(v, dtype=np.uint64)
    y = np.zeros(words(m), dtype=np.uint64)
    lda = A.shape[1] if A.shape[0] else words(k)
    _lib().gf2ref_matvec(_ptr(y), _ptr(A), lda, _ptr(v), m, k)
    return y


def pack(bits: np.ndarray, ld: int | None = None) -> np.ndarray:
    """0/1 matrix (rows x cols) -> packed uint64 words; column j is bit j&63 of word j>>6."""
    bits = np.asarray(bits, dtype=np.uint8) & 1
    rows, cols = bits.shape
    W = words(cols)
    ld = W if ld is None else ld
    out = np.zeros((rows, ld), dtype=np.uint64)
    for j in range(cols):
        out[:, j >> 6] |= bits[:, j].astype(np.uint64) << np.uint64(j & 63)
    return out


def unpack(words_: np.ndarray, cols: int) -> np.ndarray:
    words_ = np.asarray(words_, dtype=np.uint64)
    rows = words_.shape[0]
    out = np.zeros((rows, cols), dtype=np.uint8)
    for j in range(cols):
        out[:, j] = ((words_[:, j >> 6] >> np.uint64(j & 63)) & np.uint64(1)).astype(np.uint8)
    return out


def equal_packed(X: np.ndarray, Y: np.ndarray, cols: int) -> bool:
    """Compare two packed matrices on their valid bits only (padding and stride gaps ignored)."""
    W = words(cols)
    if X.shape[0] != Y.shape[0]:
        return False
    if X.shape[0] == 0 or W == 0:
        return True
    a = X[:, :W].copy()
    b = Y[:, :W].copy()
    r = cols & 63
    if r:
        mk = np.uint64((1 << r) - 1)
        a[:, W - 1] &= mk
        b[:, W - 1] &= mk
    return bool(np.array_equal(a, b))


# ---------------------------------------------------------------------------
# Method of the Four Russians (Section 3), small inputs, paper order and notation
# ---------------------------------------------------------------------------

def gray_code(kbits: int):
    """Gray code on ``kbits`` bits built as Section 3.1 describes: take the (k-1)-bit code,
    prefix every entry with 0, then the reversed list prefixed with 1, and concatenate.
    Entries are bit lists, most significant (first column in the paper's figure) first."""
    code = [[]]
    for _ in range(kbits):
        code = [[0] + c for c in code] + [[1] + c for c in reversed(code)]
    return code


def _value(bitlist) -> int:
    v = 0
    for b in bitlist:
        v = 2 * v + b
    return v


def read_bits(A_row_bits, c: int, kbits: int) -> int:
    """ReadBits(A, r, c, k) of Algorithm 1: the k bits starting at column c, first bit most
    significant.  Columns past the end of the row read as zero (the last stripe may be short)."""
    v = 0
    for b in range(kbits):
        col = c + b
        bit = int(A_row_bits[col]) if col < len(A_row_bits) else 0
        v = 2 * v + bit
    return v


def make_table(B_rows: np.ndarray, r: int, kbits: int, counter=None) -> np.ndarray:
    """MakeTable(B, r, 0, k): all 2^k linear combinations of rows r..r+k-1 of B (packed rows),
    indexed by the k-bit value read as ReadBits does.  Built along the Gray code so that each
    new entry costs one row addition (Section 3.1).  Rows of B past its end count as zero."""
    nrow, W = B_rows.shape
    T = np.zeros((1 << kbits, W), dtype=np.uint64)
    code = gray_code(kbits)
    for i in range(1, len(code)):
        prev, cur = code[i - 1], code[i]
        pos = [p for p in range(kbits) if prev[p] != cur[p]]
        assert len(pos) == 1
        src = r + pos[0]   # bit position p (from the most significant) selects row r + p
        row = B_rows[src] if src < nrow else np.zeros(W, dtype=np.uint64)
        T[_value(cur)] = T[_value(prev)] ^ row
        if counter is not None:
            counter[0] += 1
    return T


def m4rm(A_bits: np.ndarray, B_packed: np.ndarray, kbits: int, tables: int = 1, block_rows: int | None = None,
         counter=None) -> np.ndarray:
    """Algorithms 1-3 of Section 3 on small inputs.

    ``A_bits`` is the unpacked 0/1 m x l matrix (ReadBits works bit by bit), ``B_packed`` the packed
    l x n matrix; the result is packed m x n.  ``tables`` = t Gray-code tables per pass
    (Algorithm 3; t = 1 is Algorithm 1).  ``block_rows`` applies the row blocking of Algorithm 2.
    Where k (or t*k) does not divide l the last pass simply has fewer real rows of B: ReadBits
    returns zero for the missing columns and MakeTable treats the missing rows as zero.
    """
    m, l = A_bits.shape
    W = B_packed.shape[1]
    C = np.zeros((m, W), dtype=np.uint64)
    step = tables * kbits
    npass = -(-l // step) if l else 0
    blocks = [(0, m)] if not block_rows else [(s, min(m, s + block_rows)) for s in range(0, m, block_rows)]
    for (r0, r1) in blocks:
        for i in range(npass):
            Ts = [make_table(B_packed, i * step + q * kbits, kbits, counter) for q in range(tables)]
            for j in range(r0, r1):
                for q in range(tables):
                    x = read_bits(A_bits[j], i * step + q * kbits, kbits)
                    C[j] ^= Ts[q][x]
    return C


# ---------------------------------------------------------------------------
# Strassen-Winograd (Section 4, Algorithm 4)
# ---------------------------------------------------------------------------

class RingOps:
    """Ring used by ``strassen_winograd``: over GF(2) add = sub = XOR; over the integers real +/-."""

    def __init__(self, add, sub, base_mul, zeros):
        self.add, self.sub, self.base_mul, self.zeros = add, sub, base_mul, zeros


def gf2_ring():
    return RingOps(lambda x, y: x ^ y, lambda x, y: x ^ y,
                   lambda x, y: ((x.astype(np.int64) @ y.astype(np.int64)) & 1).astype(np.uint8),
                   lambda s: np.zeros(s, dtype=np.uint8))


def int_ring():
    return RingOps(lambda x, y: x + y, lambda x, y: x - y, lambda x, y: x @ y,
                   lambda s: np.zeros(s, dtype=np.int64))


def strassen_winograd(A, B, ring: RingOps, cutoff: int, odd: str = "pad", counter=None):
    """Algorithm 4 on dense (unpacked) matrices.

    Recursion stops when any dimension is at most ``cutoff`` (Section 5) and the base case is
    ``ring.base_mul``.  Odd dimensions: ``odd='pad'`` appends a zero row/column virtually
    (Section 4, padding); ``odd='peel'`` recurses on the largest even submatrices and resolves
    the rest with non-recursive products (Section 4, peeling).  ``counter`` (dict) counts
    products and additions per recursion node.
    """
    m, l = A.shape
    l2, n = B.shape
    assert l == l2
    if min(m, l, n) <= cutoff or min(m, l, n) < 2:
        if counter is not None:
            counter["base"] = counter.get("base", 0) + 1
        return ring.base_mul(A, B)
    if odd == "peel" and (m % 2 or l % 2 or n % 2):
        me, le, ne = m - m % 2, l - l % 2, n - n % 2
        C = ring.zeros((m, n))
        Cm = strassen_winograd(A[:me, :le], B[:le, :ne], ring, cutoff, odd, counter)
        if le < l:   # fix-up: the peeled inner column/row
            Cm = ring.add(Cm, ring.base_mul(A[:me, le:], B[le:, :ne]))
        C[:me, :ne] = Cm
        if ne < n:
            C[:me, ne:] = ring.base_mul(A[:me, :], B[:, ne:])
        if me < m:
            C[me:, :] = ring.base_mul(A[me:, :], B)
        return C
    if m % 2 or l % 2 or n % 2:   # virtual padding: zero rows/columns, crop the result
        Ap = ring.zeros((m + m % 2, l + l % 2))
        Bp = ring.zeros((l + l % 2, n + n % 2))
        Ap[:m, :l] = A
        Bp[:l, :n] = B
        return strassen_winograd(Ap, Bp, ring, cutoff, odd, counter)[:m, :n]
    h, g, f = m // 2, l // 2, n // 2
    A_NW, A_NE, A_SW, A_SE = A[:h, :g], A[:h, g:], A[h:, :g], A[h:, g:]
    B_NW, B_NE, B_SW, B_SE = B[:g, :f], B[:g, f:], B[g:, :f], B[g:, f:]
    add, sub = ring.add, ring.sub
    # 8 additions
    S0 = add(A_SW, A_SE)
    S1 = sub(S0, A_NW)
    S2 = sub(A_NW, A_SW)
    S3 = sub(A_NE, S1)
    T0 = sub(B_NE, B_NW)
    T1 = sub(B_SE, T0)
    T2 = sub(B_SE, B_NE)
    T3 = sub(T1, B_SW)
    rec = lambda X, Y: strassen_winograd(X, Y, ring, cutoff, odd, counter)
    # 7 recursive multiplications
    P0 = rec(A_NW, B_NW)
    P1 = rec(A_NE, B_SW)
    P2 = rec(S3, B_SE)
    P3 = rec(A_SE, T3)
    P4 = rec(S0, T0)
    P5 = rec(S1, T1)
    P6 = rec(S2, T2)
    # 7 final additions
    U0 = add(P0, P1)
    U1 = add(P0, P5)
    U2 = add(U1, P6)
    U3 = add(U1, P4)
    U4 = add(U3, P2)
    U5 = sub(U2, P3)
    U6 = add(U2, P4)
    if counter is not None:
        counter["nodes"] = counter.get("nodes", 0) + 1
        counter["adds"] = counter.get("adds", 0) + 15
        counter["products"] = counter.get("products", 0) + 7
    C = ring.zeros((m, n))
    C[:h, :f], C[:h, f:] = U0, U4       # Augment(U0, U4)
    C[h:, :f], C[h:, f:] = U5, U6       # Augment(U5, U6); Stack
    return C


# ---------------------------------------------------------------------------
# Tuning rule of Section 5
# ---------------------------------------------------------------------------

def paper_tuning(l2_bytes: int, l1_bytes: int, tables: int = 8):
    """c_s: largest power of two such that two c_s x c_s bit matrices fit in L2; b_s = c_s/2;
    k = floor(0.75 log2 b_s) - 2, lowered by one more when that makes the t tables of width
    c_s bits fit in L1 while they did not fit before.  Returns (c_s, b_s, k, table_bytes)."""
    cs = 1
    while 2 * ((2 * cs) ** 2) // 8 <= l2_bytes:
        cs *= 2
    bs = cs // 2
    k = int(math.floor(0.75 * math.log2(bs))) - 2
    table_bytes = lambda kk: tables * (1 << kk) * cs // 8
    if table_bytes(k) > l1_bytes and table_bytes(k - 1) <= l1_bytes:
        k -= 1
    return cs, bs, k, table_bytes(k)
