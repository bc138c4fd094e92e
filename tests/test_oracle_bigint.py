"""Pins of the long-integer product oracle: two's complement round trips,
hand-checked values at the word boundaries, and the product against explicit
loops over Python integers built independently of the plane layout."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import bigint


def planes_of(values, words):
    """Independent encoder: each value's bytes via int.to_bytes."""
    arr = np.array(values, dtype=object)
    out = np.zeros((words,) + arr.shape, dtype=np.uint32)
    for idx in np.ndindex(arr.shape):
        b = int(arr[idx]).to_bytes(4 * words, "little", signed=True)
        for w in range(words):
            out[(w,) + idx] = int.from_bytes(b[4 * w:4 * w + 4], "little")
    return out


def test_decode_encode_round_trip_and_boundaries():
    vals = [[0, 1, -1], [2 ** 63 - 1, -(2 ** 63), 2 ** 32], [-(2 ** 32), 12345678901234567890 // 3, -7]]
    P = planes_of(vals, 2)
    X = bigint.decode(P)
    assert [[int(v) for v in row] for row in X] == vals
    assert np.array_equal(bigint.encode(X, 2), P)
    # -1 is all ones; 2^32 has word 1 = 1
    assert P[0, 0, 2] == 0xFFFFFFFF and P[1, 0, 2] == 0xFFFFFFFF
    assert P[0, 1, 2] == 0 and P[1, 1, 2] == 1
    with pytest.raises(ValueError):
        bigint.encode(np.array([[2 ** 63]], dtype=object), 2)


def test_product_matches_explicit_loops():
    g = np.random.default_rng(5)
    m, n, l, wa, wb = 3, 4, 5, 3, 2
    A = [[int(g.integers(-2 ** 62, 2 ** 62)) * int(g.integers(1, 2 ** 30)) for _ in range(l)] for _ in range(m)]
    B = [[int(g.integers(-2 ** 62, 2 ** 62)) for _ in range(n)] for _ in range(l)]
    C = bigint.gemm(planes_of(A, wa), planes_of(B, wb))
    wc = C.shape[0]
    assert wc == bigint.words_needed(wa, wb, l)
    want = [[sum(A[i][k] * B[k][j] for k in range(l)) for j in range(n)] for i in range(m)]
    assert np.array_equal(C, planes_of(want, wc))


def test_extreme_values_fit():
    """The most negative values of both operands at every k: the largest
    product magnitude fits the word count exactly as stated."""
    wa, wb, l = 2, 3, 7
    A = [[-(2 ** (32 * wa - 1))] * l]
    B = [[-(2 ** (32 * wb - 1))] for _ in range(l)]
    C = bigint.gemm(planes_of(A, wa), planes_of(B, wb))
    assert int(bigint.decode(C)[0, 0]) == l * 2 ** (32 * (wa + wb) - 2)
