"""Pins of the exact BLAS-form oracle (alpha op(A) op(B) + beta C) against
brute force in rational arithmetic, written with explicit index loops and an
explicit complex product, and against the plain product of Eq. (1)."""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import blas, exact
from paper_1710_01839_amd import inputs


def Fr(planes, i, j) -> Fraction:
    return sum((Fraction(float(p[i, j])) for p in planes), Fraction(0))


def Fs(limbs) -> Fraction:
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def entry(planes, trans, i, p):
    """op(X)_ip read straight from storage."""
    return Fr(planes, i, p) if trans == "N" else Fr(planes, p, i)


def as_fraction(R, s):
    return np.vectorize(lambda v: Fraction(int(v), 1 << s), otypes=[object])(R)


def stored(rows, cols, trans, seed):
    r, c = (rows, cols) if trans == "N" else (cols, rows)
    return inputs.dd_illcond(r, c, seed_offset=seed, kmax=8)


SCALARS = [((1.0, 0.0), (0.0, 0.0)),
           ((-2.5, 2.0 ** -60), (0.75, -2.0 ** -57)),
           ((0.0, 0.0), (3.0, 2.0 ** -53)),
           ((1.0 / 3, 1.0 / 3 * 2.0 ** -54), (0.0, 0.0))]


@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("sc", range(len(SCALARS)))
def test_real_form_matches_brute_force(ta, tb, sc):
    m, n, k = 3, 4, 5
    alpha, beta = SCALARS[sc]
    A = stored(m, k, ta, 1)
    B = stored(k, n, tb, 2)
    C = inputs.dd_illcond(m, n, seed_offset=3, kmax=8)
    R, mab, mc, s = blas.rgemm_exact(ta, tb, alpha, A, B, beta, C)
    got = as_fraction(R, s)
    a, b = Fs(alpha), Fs(beta)
    for i in range(m):
        for j in range(n):
            dot = sum(entry(A, ta, i, p) * entry(B, tb, p, j) for p in range(k))
            want = a * dot + b * Fr(C, i, j)
            assert got[i, j] == want
            mag = abs(a) * sum(abs(entry(A, ta, i, p)) * abs(entry(B, tb, p, j)) for p in range(k))
            assert Fraction(int(mab[i, j]), 1 << s) == mag
            assert Fraction(int(mc[i, j]), 1 << s) == abs(b) * abs(Fr(C, i, j))


def test_real_form_reduces_to_the_plain_product():
    A = inputs.qd_uniform(6, 7, seed_offset=4)
    B = inputs.qd_uniform(7, 5, seed_offset=5)
    C = inputs.qd_uniform(6, 5, seed_offset=6)
    R, _, _, s = blas.rgemm_exact("N", "N", (1.0, 0.0, 0.0, 0.0), A, B, (0.0,) * 4, C)
    P, sp = exact.matmul_exact(A, B)
    assert s >= sp and (R == P * (1 << (s - sp))).all()


def test_real_form_ignores_unread_operands():
    m, n, k = 3, 3, 4
    A = stored(m, k, "N", 1)
    B = stored(k, n, "N", 2)
    C = inputs.dd_uniform(m, n, seed_offset=3)
    Cnan = (np.full((m, n), np.nan), np.zeros((m, n)))
    # beta == 0: C is not read
    R1, _, _, s1 = blas.rgemm_exact("N", "N", (2.0, 0.0), A, B, (0.0, 0.0), Cnan)
    R2, _, _, s2 = blas.rgemm_exact("N", "N", (2.0, 0.0), A, B, (0.0, 0.0), C)
    assert (as_fraction(R1, s1) == as_fraction(R2, s2)).all()
    # alpha == 0: the product is not formed; k == 0: beta C
    Anan = (np.full((m, k), np.nan), np.zeros((m, k)))
    R3, _, _, s3 = blas.rgemm_exact("N", "N", (0.0, 0.0), Anan, B, (0.5, 0.0), C)
    R4, _, _, s4 = blas.rgemm_exact("N", "N", (7.0, 0.0), (np.zeros((m, 0)),) * 2,
                                    (np.zeros((0, n)),) * 2, (0.5, 0.0), C)
    half = np.vectorize(lambda i, j: Fr(C, i, j) / 2, otypes=[object])(*np.indices((m, n)))
    assert (as_fraction(R3, s3) == half).all() and (as_fraction(R4, s4) == half).all()


def cmul(x, y):
    return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])


def centry(Z, trans, i, p):
    re = entry(Z[0], trans, i, p)
    im = entry(Z[1], trans, i, p)
    return (re, -im) if trans == "C" else (re, im)


@pytest.mark.parametrize("ta,tb", list(itertools.product("NTC", "NTC")))
def test_complex_form_matches_brute_force(ta, tb):
    m, n, k = 2, 3, 4
    alpha = ((0.75, 2.0 ** -56), (-1.5, 0.0))
    beta = ((-0.5, 0.0), (2.0, -2.0 ** -55))
    A = (stored(m, k, ta, 11), stored(m, k, ta, 12))
    B = (stored(k, n, tb, 13), stored(k, n, tb, 14))
    C = (inputs.dd_uniform(m, n, seed_offset=15), inputs.dd_uniform(m, n, seed_offset=16))
    Rr, Ri, mab, mc, s = blas.zgemm_exact(ta, tb, alpha, A, B, beta, C)
    gr, gi = as_fraction(Rr, s), as_fraction(Ri, s)
    a = (Fs(alpha[0]), Fs(alpha[1]))
    b = (Fs(beta[0]), Fs(beta[1]))
    for i in range(m):
        for j in range(n):
            acc = (Fraction(0), Fraction(0))
            for p in range(k):
                t = cmul(centry(A, ta, i, p), centry(B, tb, p, j))
                acc = (acc[0] + t[0], acc[1] + t[1])
            x = cmul(a, acc)
            y = cmul(b, (Fr(C[0], i, j), Fr(C[1], i, j)))
            assert gr[i, j] == x[0] + y[0]
            assert gi[i, j] == x[1] + y[1]
            # the stated magnitudes bound both parts of each term
            ma = Fraction(int(mab[i, j]), 1 << s)
            mcc = Fraction(int(mc[i, j]), 1 << s)
            assert max(abs(x[0]), abs(x[1])) <= ma and max(abs(y[0]), abs(y[1])) <= mcc


def test_conjugation_changes_the_result():
    m, n, k = 2, 2, 3
    A = (stored(m, k, "T", 21), stored(m, k, "T", 22))
    B = (stored(k, n, "N", 23), stored(k, n, "N", 24))
    C = (np.zeros((m, n)),) * 2, (np.zeros((m, n)),) * 2
    one, zero = ((1.0, 0.0), (0.0, 0.0)), ((0.0, 0.0), (0.0, 0.0))
    Rt = blas.zgemm_exact("T", "N", one, A, B, zero, C)
    Rc = blas.zgemm_exact("C", "N", one, A, B, zero, C)
    assert not (Rt[0] == Rc[0]).all() and not (Rt[1] == Rc[1]).all()


def test_error_over_bound_measures_exactly():
    m, n, k = 2, 2, 2
    A = stored(m, k, "N", 31)
    B = stored(k, n, "N", 32)
    C = inputs.dd_uniform(m, n, seed_offset=33)
    R, mab, mc, s = blas.rgemm_exact("N", "N", (1.0, 0.0), A, B, (1.0, 0.0), C)
    val = Fraction(int(R[0, 0]), 1 << s)
    hi = float(val)
    lo = float(val - Fraction(hi))
    out = [np.array([[hi, 0.0], [0.0, 0.0]]), np.array([[lo, 0.0], [0.0, 0.0]])]
    for idx in [(0, 1), (1, 0), (1, 1)]:
        v = Fraction(int(R[idx]), 1 << s)
        out[0][idx] = float(v)
        out[1][idx] = float(v - Fraction(float(v)))
    # round to nearest in two limbs: error <= 2^-106 |value| <= 2^-106 (mab + mc)
    r = blas.error_over_bound(tuple(out), R, mab, mc, s, 1, 1, -106)
    assert r <= 1.0
    # a deliberate one-ulp change of a lower limb is visible
    out[1][0, 0] = np.nextafter(out[1][0, 0], np.inf) if out[1][0, 0] != 0 else 2.0 ** -200
    assert blas.error_over_bound(tuple(out), R, mab, mc, s, 1, 1, -106) > r
