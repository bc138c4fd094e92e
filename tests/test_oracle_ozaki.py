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
            v = sum(Fraction(int(D[s][i, k]), 256 ** (s + 1)) for s in range(S))
            assert v * Fraction(2) ** int(e[i] + 2) == Fraction(float(A[i, k]))
            assert -64 <= int(D[0][i, k]) <= 64
            assert D[0][i, k] == 0 or (D[0][i, k] > 0) == (A[i, k] > 0)
            for s in range(S):
                assert -128 <= int(D[s][i, k]) <= 127
    # one slice fewer leaves a remainder somewhere
    D2, y2 = ozaki.split_rows(A, e, S - 1)
    assert np.any(y2 != 0.0) and np.all(np.abs(y2) < 1.0) and np.all(y2 * A >= 0.0)


def test_signed_bytes_carry():
    """Truncated digits 31, 255, 255, 252 (value 31/256 + 255/256^2 +
    255/256^3 + 252/256^4) become 32, 0, 0, -4, and their negatives -32, 0,
    0, 4: the same values in signed bytes."""
    F = [np.array([31, -31]), np.array([255, -255]), np.array([255, -255]), np.array([252, -252])]
    D = ozaki.signed_bytes(F)
    assert [int(d[0]) for d in D] == [32, 0, 0, -4] and [int(d[1]) for d in D] == [-32, 0, 0, 4]
    g = np.random.default_rng(5)
    sign = np.where(g.random(200) < 0.5, -1, 1)
    F = [sign * g.integers(0, 64, 200)] + [sign * g.integers(0, 256, 200) for _ in range(6)]
    D = ozaki.signed_bytes(F)
    for j in range(200):
        assert sum(Fraction(int(F[s][j]), 256 ** s) for s in range(7)) == \
            sum(Fraction(int(D[s][j]), 256 ** s) for s in range(7))
    assert all(-128 <= int(x) <= 127 for d in D[1:] for x in d)
    assert all(-64 <= int(x) <= 64 for x in D[0])


def test_single_slice_integer_product_exact():
    """Integer entries in [-63, 63] with every row / column maximum >= 32
    (scale 2^6, so 256 y = x / 2^0 ... one digit of weight 2^0): one slice
    holds them exactly, so the result is exactly AB."""
    g = np.random.default_rng(3)
    A = g.integers(-63, 64, size=(9, 40)).astype(float)
    B = g.integers(-63, 64, size=(40, 7)).astype(float)
    A[:, 0] = 63.0
    B[0, :] = -40.0
    assert ozaki.slices_exact(A, B) == 1
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
    """hi + lo = 2^(e + 2) sum_s D_s 256^-s once S covers the lowest set bit
    of either limb; digits stay signed bytes; one slice fewer leaves a
    nonzero remainder (the count is the smallest exact one)."""
    hi, lo = inputs.dd_uniform(6, 9, 5)
    e = ozaki.row_exponents(hi)
    S = ozaki.slices_exact((hi, lo), (hi.T.copy(), lo.T.copy()))
    assert S >= 14                      # ~106 bits below the row scale
    D, rem = ozaki.split_rows_dd(hi, lo, e, S)
    for i in range(6):
        for k in range(9):
            v = sum(Fraction(int(D[s][i, k]), 256 ** (s + 1)) for s in range(S))
            assert v * Fraction(2) ** int(e[i] + 2) == Fraction(float(hi[i, k])) + Fraction(float(lo[i, k]))
            assert rem[i, k] == 0
            assert all(-128 <= int(D[s][i, k]) <= 127 for s in range(S))
    need_rows = max(ozaki.slices_needed_rows(hi, e), ozaki.slices_needed_rows(lo, e))
    _, rem2 = ozaki.split_rows_dd(hi, lo, e, need_rows - 1)
    assert any(r != 0 for r in rem2.flat)


def test_dd_split_signed_digits_worked_example():
    """hi = 1/2, lo = -2^-60 (value just below 1/2, e = 0): y = 1/8 - 2^-62,
    256 y = 32 - 2^-54 gives the digit 31 and remainder 1 - 2^-54, which
    grows by 256 per step (digits 255) until
    256 (1 - 2^-6) = 252; the carry from the bottom turns 31, 255 x 6, 252
    into 32, 0 x 6, -4 (4 256^-8 = 2^-62)."""
    hi = np.array([[0.5]])
    lo = np.array([[-2.0 ** -60]])
    D, rem = ozaki.split_rows_dd(hi, lo, np.array([0]), 10)
    got = [int(D[s][0, 0]) for s in range(10)]
    assert got == [32, 0, 0, 0, 0, 0, 0, -4, 0, 0]
    assert rem[0, 0] == 0
    assert ozaki.slices_exact((hi, lo), (hi.copy(), lo.copy())) == 8
    # the mirror image: truncation toward zero gives the negated digits
    D, rem = ozaki.split_rows_dd(-hi, -lo, np.array([0]), 10)
    assert [int(D[s][0, 0]) for s in range(10)] == [-32, 0, 0, 0, 0, 0, 0, 4, 0, 0]


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


@pytest.mark.parametrize("S", [2, 4, 6])
def test_triangle_bound_term_is_attained(S):
    """y = 40/256 + sum_{s=2}^{S-1} 127/256^s + 128/256^S (x = 4 y in [1/2, 1),
    scale 2^0): truncated digits 40, 127, ..., 127, 128 carry into signed bytes
    41, -128, ..., -128, so every pair the triangle drops is (-128)^2 =
    2^14, the per-pair maximum of the bound: the error of x*x equals the
    dropped-diagonal term of the a-priori bound, pair count included."""
    y = Fraction(40, 256) + sum(Fraction(127, 256 ** s) for s in range(2, S)) + Fraction(128, 256 ** S)
    x = 4 * y
    assert float(x) == x                       # 8S <= 48 bits: exact in binary64
    A = np.array([[float(x)]])
    D, _ = ozaki.split_rows(A, ozaki.row_exponents(A), S)
    assert [int(d[0, 0]) for d in D] == [41] + [-128] * (S - 1)
    (_, _), (N, E0) = ozaki.ozaki_dd(A, A.copy(), S, "triangle")
    err = x * x - ozaki.to_fraction(N, E0, (0, 0))
    dropped = sum(Fraction(2 ** 14 * 16, 256 ** (s + t)) for s in range(1, S + 1)
                  for t in range(1, S + 1) if s + t > S + 1)
    assert err == dropped
    term = ozaki.apriori_unit(S, "triangle") - ozaki.apriori_unit(S, "all")
    assert abs(float(dropped) - term) <= 2.0 ** -50 * term


def test_qd_split_reduces_to_dd_split():
    """Quad-double values whose limbs 2 and 3 are zero split digit for digit
    like the double-double values of their first two limbs."""
    hi, lo = inputs.dd_uniform(5, 7, 8)
    e = ozaki.row_exponents(hi)
    S = ozaki.slices_exact((hi, lo), (hi.T.copy(), lo.T.copy()))
    D1, r1 = ozaki.split_rows_dd(hi, lo, e, S)
    D2, r2 = ozaki.split_rows_limbs((hi, lo, np.zeros_like(hi), np.zeros_like(hi)), e, S)
    assert all(np.array_equal(a, b) for a, b in zip(D1, D2))
    assert all(x == y for x, y in zip(r1.flat, r2.flat))


def test_qd_split_and_product_exact():
    """Quad-double inputs: the exact slice count (about 212 bits below the
    row scale, so 27 or more slices) reconstructs every element, and the
    combination is exactly AB (against the integer definition)."""
    A = inputs.qd_uniform(4, 6, 9)
    B = inputs.qd_uniform(6, 3, 10)
    S = ozaki.slices_exact(A, B)
    assert S >= 27
    e = ozaki.row_exponents(A[0])
    D, rem = ozaki.split_rows_limbs(A, e, S)
    for i in range(4):
        for k in range(6):
            v = sum(Fraction(int(D[s][i, k]), 256 ** (s + 1)) for s in range(S))
            assert v * Fraction(2) ** int(e[i] + 2) == sum(Fraction(float(x[i, k])) for x in A)
            assert rem[i, k] == 0
    C, (N, E0) = ozaki.ozaki_dd(A, B, S, "all", out_limbs=4)
    Ci, s = exact.matmul_exact(A, B)
    for idx in np.ndindex(C[0].shape):
        assert ozaki.to_fraction(N, E0, idx) == Fraction(int(Ci[idx]), 2 ** s)
