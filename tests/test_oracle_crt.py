"""Pins of the residue (CRT) form of the split product: the moduli, the
reconstruction on hand-checked and exhaustive small cases, the integer images
against the digit form, the product against exact integer arithmetic, and
the correctly rounded result under exact slicing."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from oracle import crt, exact, ozaki
from paper_1710_01839_amd import inputs


def test_moduli_are_pairwise_coprime_and_largest_first():
    mods = crt.moduli()
    assert mods[:6] == [256, 255, 253, 251, 247, 241]
    assert len(mods) == 49 and mods == sorted(mods, reverse=True)
    for i, p in enumerate(mods):
        for q in mods[:i]:
            assert math.gcd(p, q) == 1
    # every skipped integer in (mods[-1], 256] shares a factor with a kept one
    for x in range(mods[-1] + 1, 257):
        if x not in mods:
            assert any(math.gcd(x, p) > 1 for p in mods if p > x)
    assert abs(sum(math.log2(p) for p in mods) - 341.9) < 0.05


def test_crt_hand_example_and_exhaustive_small_range():
    # X = 3 mod 5, X = 2 mod 7: X = 23, centred in [-17.5, 17.5): -12
    r = crt.crt([np.array([3], dtype=object), np.array([2], dtype=object)], [5, 7])
    assert r[0] == -12
    mods = [4, 9, 5]
    P = 180
    xs = list(range(-P // 2, P // 2))
    res = [np.array([x % p for x in xs], dtype=object) for p in mods]
    assert list(crt.crt(res, mods)) == xs


def test_images_are_the_digit_sums():
    A = inputs.dd_illcond(5, 9, seed_offset=70, kmax=10)
    e = ozaki.row_exponents(A[0])
    for S in (1, 3, 8, 17):
        Ai = crt.images_rows(A, e, S)
        D, _ = ozaki.split_rows_limbs(A, e, S)
        want = sum(np.asarray(D[s], dtype=object) * 256 ** (S - 1 - s) for s in range(S))
        assert (Ai == want).all()
        assert all(abs(int(v)) < 2 ** (8 * S - 2) for v in Ai.flat)


def test_product_is_the_exact_integer_product():
    A = inputs.dd_uniform(6, 11, seed_offset=71)
    B = inputs.dd_uniform(11, 4, seed_offset=72)
    e, f = ozaki.row_exponents(A[0]), ozaki.col_exponents(B[0])
    for S in (2, 7, 17):
        C, X, _ = crt.crt_product(A, B, S)
        want = crt.images_rows(A, e, S).dot(crt.images_cols(B, f, S))
        assert (X == want).all()
        assert max(abs(int(v)) for v in X.flat) < 2 ** (crt.product_bits(S, 11) - 1)


def test_exact_slicing_gives_the_correctly_rounded_product():
    for A, B in ((inputs.dd_uniform(5, 13, 73), inputs.dd_uniform(13, 6, 74)),
                 (inputs.dd_illcond(4, 9, 75, kmax=12), inputs.dd_illcond(9, 5, 76, kmax=12))):
        S = ozaki.slices_exact(A, B)
        C, _, _ = crt.crt_product(A, B, S)
        P, s = exact.matmul_exact(A, B)
        for idx in np.ndindex(P.shape):
            want = exact.round_to_limbs(Fraction(int(P[idx]), 1 << s), 2)
            assert (C[0][idx], C[1][idx]) == tuple(want)


def test_too_few_moduli_fail():
    """A product that needs three moduli is wrong with two."""
    A = (np.full((1, 64), 0.99), np.zeros((1, 64)))
    B = (np.full((64, 1), 0.99), np.zeros((64, 1)))
    need = crt.moduli_for_bits(crt.product_bits(1, 64))
    assert need == 3
    _, X, _ = crt.crt_product(A, B, 1)
    assert X[0, 0] == 64 * 63 * 63
    _, X2, _ = crt.crt_product(A, B, 1, N=2)
    assert X2[0, 0] != X[0, 0]
