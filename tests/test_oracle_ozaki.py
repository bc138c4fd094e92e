"""Pins of the split-precision oracle: exact reconstruction of the digit
planes, digit range and sign, exact integer special cases, agreement with
the exact product when nothing is truncated, and the a-priori truncation
bound."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact, ozaki
from paper_1710_01839_amd import inputs


def test_exponents():
    A = np.array([[0.5, -0.25], [0.0, 0.0], [3.0, 1.0], [-1.0, 0.75]])
    assert list(ozaki.row_exponents(A)) == [0, 0, 2, 1]      # max < 2^e, zero row -> 0


def test_split_reconstructs_and_digits_in_range():
    A = inputs.fp64_wide(20, 30, 0)
    e = ozaki.row_exponents(A)
    S = ozaki.slices_needed_rows(A, e)
    assert 10 <= S <= 30
    D, y = ozaki.split_rows(A, e, S)
    assert np.all(y == 0.0)
    for i in range(20):
        for k in range(30):
            v = sum(Fraction(int(D[s][i, k]), 128 ** (s + 1)) for s in range(S))
            assert v * Fraction(2) ** int(e[i]) == Fraction(float(A[i, k]))
            for s in range(S):
                d = int(D[s][i, k])
                assert -127 <= d <= 127
                assert d == 0 or (d > 0) == (A[i, k] > 0)
    # one slice fewer leaves a remainder somewhere
    D2, y2 = ozaki.split_rows(A, e, S - 1)
    assert np.any(y2 != 0.0)


def test_single_slice_integer_product_exact():
    """Integer entries in [-127, 127] with every row / column maximum >= 64:
    one slice holds them exactly, so the result is exactly AB."""
    g = np.random.default_rng(3)
    A = g.integers(-127, 128, size=(9, 40)).astype(float)
    B = g.integers(-127, 128, size=(40, 7)).astype(float)
    A[:, 0] = 127.0
    B[0, :] = -100.0
    (hi, lo), (N, E0) = ozaki.ozaki_dd(A, B, 1)
    want = A.astype(np.int64) @ B.astype(np.int64)
    for idx in np.ndindex(want.shape):
        assert ozaki.to_fraction(N, E0, idx) == int(want[idx])
    assert np.array_equal(hi, want.astype(float))


def test_exact_slices_give_exact_product():
    A = inputs.fp64_wide(6, 25, 1)
    B = inputs.fp64_wide(25, 5, 2)
    S = ozaki.slices_exact(A, B)
    (hi, lo), (N, E0) = ozaki.ozaki_dd(A, B, S, "all")
    Ci, s = exact.matmul_exact((A,), (B,))
    for idx in np.ndindex(hi.shape):
        assert ozaki.to_fraction(N, E0, idx) == Fraction(int(Ci[idx]), 2 ** s)


@pytest.mark.parametrize("mode", ["all", "triangle"])
@pytest.mark.parametrize("S", [3, 6, 10])
def test_truncated_within_apriori_bound(S, mode):
    A = inputs.fp64_wide(8, 50, 3)
    B = inputs.fp64_wide(50, 6, 4)
    (hi, lo), (N, E0) = ozaki.ozaki_dd(A, B, S, mode)
    Ci, s = exact.matmul_exact((A,), (B,))
    bound = ozaki.apriori_bound(A, B, S, mode)
    worst = 0.0
    for idx in np.ndindex(hi.shape):
        err = abs(ozaki.to_fraction(N, E0, idx) - Fraction(int(Ci[idx]), 2 ** s))
        assert err <= Fraction(float(bound[idx]))
        worst = max(worst, float(err) / bound[idx])
    assert worst > 0          # truncation does lose something at these S


def test_pair_sets():
    assert len(ozaki.pairs(5, "all")) == 25
    assert len(ozaki.pairs(5, "triangle")) == 15
    assert all(s + t <= 6 for s, t in ozaki.pairs(5, "triangle"))


def test_dd_split_reduces_to_fp64_split():
    """lo = 0: the double-double split is the FP64 split, digit for digit."""
    A = inputs.fp64_wide(7, 11, 4)
    e = ozaki.row_exponents(A)
    D1, y1 = ozaki.split_rows(A, e, 9)
    D2, r2 = ozaki.split_rows_dd(A, np.zeros_like(A), e, 9)
    for s in range(9):
        assert np.array_equal(D1[s], D2[s])
    for idx in np.ndindex(A.shape):
        assert r2[idx] == Fraction(float(y1[idx]))


def test_dd_split_reconstructs_exactly():
    """hi + lo = 2^e sum_s D_s 128^-s once S covers the lowest set bit of
    either limb; digits stay in [-127, 127]; one slice fewer leaves a
    nonzero remainder (the count is the smallest exact one)."""
    hi, lo = inputs.dd_uniform(6, 9, 5)
    e = ozaki.row_exponents(hi)
    S = ozaki.slices_exact((hi, lo), (hi.T.copy(), lo.T.copy()))
    assert S >= 16                      # ~106 bits below the row scale
    D, rem = ozaki.split_rows_dd(hi, lo, e, S)
    for i in range(6):
        for k in range(9):
            v = sum(Fraction(int(D[s][i, k]), 128 ** (s + 1)) for s in range(S))
            assert v * Fraction(2) ** int(e[i]) == Fraction(float(hi[i, k])) + Fraction(float(lo[i, k]))
            assert rem[i, k] == 0
            assert all(-127 <= int(D[s][i, k]) <= 127 for s in range(S))
    need_rows = max(ozaki.slices_needed_rows(hi, e), ozaki.slices_needed_rows(lo, e))
    _, rem2 = ozaki.split_rows_dd(hi, lo, e, need_rows - 1)
    assert any(r != 0 for r in rem2.flat)


def test_dd_split_signed_digits_worked_example():
    """hi = 1/2, lo = -2^-60 (value just below 1/2, e = 0): 128 r_0 =
    64 - 2^-53 rounds to 64, so D_1 = 64 and the remainder r_1 = -2^-53 is
    carried by a negative digit: r grows by 128 per step until
    128 r_8 = -2^-53 128^8 = -8, so D_9 = -8 (8 128^-9 = 2^-60)."""
    hi = np.array([[0.5]])
    lo = np.array([[-2.0 ** -60]])
    D, rem = ozaki.split_rows_dd(hi, lo, np.array([0]), 10)
    got = [int(D[s][0, 0]) for s in range(10)]
    assert got == [64, 0, 0, 0, 0, 0, 0, 0, -8, 0]
    assert rem[0, 0] == 0


def test_dd_exact_slices_give_exact_product():
    """Double-double inputs with the exact slice count: the combination is
    exactly A B (the exact product of the limb sums)."""
    A = inputs.dd_uniform(5, 12, 6)
    B = inputs.dd_uniform(12, 4, 7)
    S = ozaki.slices_exact(A, B)
    (hi, lo), (N, E0) = ozaki.ozaki_dd(A, B, S, "all")
    Ci, s = exact.matmul_exact(A, B)
    for idx in np.ndindex(hi.shape):
        assert ozaki.to_fraction(N, E0, idx) == Fraction(int(Ci[idx]), 2 ** s)


@pytest.mark.parametrize("S", [2, 4, 7])
def test_triangle_bound_term_is_attained(S):
    """x = sum_{s<=S} 127 2^-7s (every digit 127, no remainder): the triangle
    drops exactly the pairs s + t > S + 1, so the error of x*x equals the
    dropped-diagonal term of the a-priori bound, pair count included."""
    x = sum(Fraction(127, 128 ** s) for s in range(1, S + 1))
    assert float(x) == x                       # 7S <= 49 bits: exact in binary64
    A = np.array([[float(x)]])
    (_, _), (N, E0) = ozaki.ozaki_dd(A, A.copy(), S, "triangle")
    err = x * x - ozaki.to_fraction(N, E0, (0, 0))
    dropped = sum(Fraction(127 * 127, 128 ** (s + t)) for s in range(1, S + 1)
                  for t in range(1, S + 1) if s + t > S + 1)
    assert err == dropped
    term = ozaki.apriori_unit(S, "triangle") - ozaki.apriori_unit(S, "all")
    assert abs(float(dropped) - term) <= 2.0 ** -50 * term
