"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's checks.

This module generates bits; it does none of the multiplication's arithmetic.
Everything is counter-based so that any row or word can be regenerated alone.

Generator: splitmix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; finaliser constants as published by Vigna).
Each matrix gets its own stream key, ``key = splitmix64(seed ^ splitmix64(tag))``.

* Bernoulli(1/2) entries: word ``w`` of row ``r`` is ``splitmix64(key + r*W + w)``
  where ``W = ceil(cols / 64)``.
* Bernoulli(p) entries: bit ``j`` of row ``r`` is set iff
  ``splitmix64(key + r*64*W + j) >> 32 < floor(p * 2**32)``.

The paper times products of random dense square matrices (Section 6); it names
no dataset, so these synthetic matrices are the whole workload.

Layout (the library's ABI): row-major, 64 entries per uint64 word, column ``j``
of a row is bit ``j & 63`` of word ``j >> 6``; ``ld`` words per row with
``ld >= ceil(cols/64)``.  Bits at columns ``>= cols`` of the last word of a row
are padding and are zero unless a caller asks for garbage there.
"""
from __future__ import annotations

import math
import numpy as np

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)
TAG_A, TAG_B, TAG_X, TAG_C = 1, 2, 3, 4


def splitmix64(x):
    """splitmix64 finaliser applied to x + golden gamma; works on numpy uint64 arrays or ints."""
    scalar = not isinstance(x, np.ndarray)
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return int(z) if scalar else z


def stream_key(seed: int, tag: int) -> int:
    return splitmix64((int(seed) ^ splitmix64(int(tag))) & 0xFFFFFFFFFFFFFFFF)


def words_per_row(cols: int) -> int:
    return (int(cols) + 63) // 64


def tail_mask(cols: int) -> np.uint64:
    """Mask of the valid bits in the last word of a row with ``cols`` columns."""
    r = int(cols) & 63
    return np.uint64(0xFFFFFFFFFFFFFFFF if r == 0 else (1 << r) - 1)


def empty(rows: int, cols: int, ld: int | None = None) -> np.ndarray:
    W = words_per_row(cols)
    ld = W if ld is None else int(ld)
    assert ld >= W
    return np.zeros((int(rows), max(ld, 0)), dtype=np.uint64)


def uniform(seed: int, tag: int, rows: int, cols: int, ld: int | None = None,
            row0: int = 0, chunk_rows: int = 1 << 16) -> np.ndarray:
    """Bernoulli(1/2) bits, padding zero; rows ``row0 .. row0+rows`` of the stream."""
    W = words_per_row(cols)
    out = empty(rows, cols, ld)
    if rows == 0 or W == 0:
        return out
    key = np.uint64(stream_key(seed, tag))
    m = tail_mask(cols)
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        idx = (np.arange(row0 + r0, row0 + r1, dtype=np.uint64)[:, None] * np.uint64(W)
               + np.arange(W, dtype=np.uint64)[None, :])
        with np.errstate(over="ignore"):
            blk = splitmix64(key + idx)
        blk[:, W - 1] &= m
        out[r0:r1, :W] = blk
    return out


def bernoulli(seed: int, tag: int, rows: int, cols: int, p: float, ld: int | None = None,
              row0: int = 0) -> np.ndarray:
    """Bernoulli(p) bits per entry, stored dense; padding zero."""
    if p == 0.5:
        # Same law, cheaper: one draw per word.  Kept as the p = 1/2 definition.
        return uniform(seed, tag, rows, cols, ld, row0)
    W = words_per_row(cols)
    out = empty(rows, cols, ld)
    if rows == 0 or W == 0:
        return out
    key = np.uint64(stream_key(seed, tag))
    thr = np.uint64(int(math.floor(p * 2 ** 32)))
    shifts = np.arange(64, dtype=np.uint64)
    chunk = max(1, (1 << 22) // max(1, 64 * W))
    for r0 in range(0, rows, chunk):
        r1 = min(rows, r0 + chunk)
        base = np.arange(row0 + r0, row0 + r1, dtype=np.uint64)[:, None, None] * np.uint64(64 * W)
        j = (np.arange(W, dtype=np.uint64)[None, :, None] * np.uint64(64) + shifts[None, None, :])
        with np.errstate(over="ignore"):
            draws = splitmix64(key + base + j)
        bits = ((draws >> np.uint64(32)) < thr)
        valid = (j < np.uint64(cols))
        bits &= valid
        words = (bits.astype(np.uint64) << shifts[None, None, :]).sum(axis=2, dtype=np.uint64)
        out[r0:r1, :W] = words
    return out


def garbage_padding(mat: np.ndarray, cols: int, seed: int = 99) -> np.ndarray:
    """Return a copy with random bits in the padding of each row's last word and in the
    stride gap words.  A correct consumer ignores all of them."""
    out = mat.copy()
    rows, ld = out.shape
    W = words_per_row(cols)
    if rows == 0 or ld == 0:
        return out
    key = np.uint64(stream_key(seed, 0xBAD))
    with np.errstate(over="ignore"):
        noise = splitmix64(key + np.arange(rows * ld, dtype=np.uint64)).reshape(rows, ld)
    if W > 0:
        m = tail_mask(cols)
        out[:, W - 1] = (out[:, W - 1] & m) | (noise[:, W - 1] & ~m)
    if ld > W:
        out[:, W:] = noise[:, W:]
    return out


def log_uniform_dims(seed: int, tag: int, count: int, lo: int = 64, hi: int = 4096, ndim: int = 3) -> np.ndarray:
    """``count`` x ``ndim`` integer sizes, each floor(lo * (hi/lo)**u) with u ~ U[0,1) from splitmix64."""
    key = np.uint64(stream_key(seed, tag))
    with np.errstate(over="ignore"):
        draws = splitmix64(key + np.arange(count * ndim, dtype=np.uint64))
    u = (draws >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    vals = np.floor(lo * (hi / lo) ** u).astype(np.int64)
    return np.clip(vals, lo, hi - 1).reshape(count, ndim)


def log_uniform_p(seed: int, tag: int, count: int, lo: float = 0.01, hi: float = 0.5) -> np.ndarray:
    key = np.uint64(stream_key(seed, tag))
    with np.errstate(over="ignore"):
        draws = splitmix64(key + np.arange(count, dtype=np.uint64))
    u = (draws >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    return lo * (hi / lo) ** u
