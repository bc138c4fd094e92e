"""Exact product of matrices of long integers (the fixed-point analog of the
paper's arbitrary-precision runs), written out plainly.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

The paper measures C = AB of Eq. (1) with MPFR numbers of 128 to 2048 bits.
The GPU analog computes the product of integer matrices exactly: every entry
is a two's complement integer of `words` 32-bit words, stored as word planes
(plane w holds word w of every entry, least significant first).  A fixed-
point number x 2^-f is its integer x; the product's scale is 2^-(fa + fb).
This module decodes the planes into Python integers, multiplies with
unbounded integers (no rounding anywhere) and encodes the result.
"""
from __future__ import annotations

import numpy as np


def decode(planes: np.ndarray) -> np.ndarray:
    """planes: uint32 array (words, rows, cols).  Returns an object array of
    Python ints (two's complement of 32 * words bits)."""
    words = planes.shape[0]
    out = np.zeros(planes.shape[1:], dtype=object)
    for w in range(words):
        out = out + planes[w].astype(object) * (1 << (32 * w))
    top = 1 << (32 * words)
    half = top >> 1
    return np.vectorize(lambda v: v - top if v >= half else v, otypes=[object])(out)


def encode(X: np.ndarray, words: int) -> np.ndarray:
    """Object array of ints -> uint32 planes (words, rows, cols), two's
    complement; every value must fit."""
    lo, hi = -(1 << (32 * words - 1)), (1 << (32 * words - 1)) - 1
    flat = [int(v) for v in X.flat]
    if flat and (min(flat) < lo or max(flat) > hi):
        raise ValueError("value does not fit the word count")
    mask = (1 << (32 * words)) - 1
    out = np.zeros((words,) + X.shape, dtype=np.uint32)
    for idx in np.ndindex(X.shape):
        v = int(X[idx]) & mask
        for w in range(words):
            out[(w,) + idx] = (v >> (32 * w)) & 0xFFFFFFFF
    return out


def words_needed(words_a: int, words_b: int, l: int) -> int:
    """Words that hold every possible entry of the product: |a| <= 2^(32 wa - 1),
    |b| <= 2^(32 wb - 1), so |c| <= l 2^(32 (wa + wb) - 2)."""
    bits = 32 * (words_a + words_b) - 2 + max(l, 1).bit_length() + 1
    return -(-bits // 32)


def gemm(A_planes: np.ndarray, B_planes: np.ndarray, words_c: int | None = None) -> np.ndarray:
    """Exact C = A B as word planes of words_c words (default: enough for any
    product of these word counts)."""
    A, B = decode(A_planes), decode(B_planes)
    l = A.shape[1]
    if words_c is None:
        words_c = words_needed(A_planes.shape[0], B_planes.shape[0], l)
    return encode(A.dot(B), words_c)
