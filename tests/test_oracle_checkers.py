"""Pins of the oracle's checkers: the functions every parity verdict passes
through.

  cref.exact_diff        exact difference of two multi-limb matrices, rounded
                         once (every full-matrix GPU check);
  exact.entries_exact    exact c_ij and (|A||B|)_ij at sampled entries (the
                         large-size GPU checks);
  exact.error_ratios     the componentwise ratio |C - AB|_ij / (l 2^u (|A||B|)_ij);
  tests/helpers.py       error_ratio_full, normwise_ratio, sampled_errors.

Each is compared with brute force written here in Python Fractions (explicit
loops over limbs and k; Python's int / int division is correctly rounded), on
DD and QD data with heavy cancellation and wide exponent ranges, and each must
report a planted change of one unit in the last place of a lower limb.  A
checker that dropped a limb, a term or a sign would fail one of these.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from paper_1710_01839_amd import inputs
from tests import helpers


def F(x) -> Fraction:
    return Fraction(float(x))


def value(planes, idx) -> Fraction:
    total = Fraction(0)
    for p in planes:
        total += F(p[idx])
    return total


def nearest(q: Fraction) -> float:
    """The double nearest to q (ties to even), by correctly rounded int / int."""
    return q.numerator / q.denominator if q != 0 else 0.0


def nudge(planes, limb, idx, ulps=1):
    """Copy of `planes` with limb `limb` at idx moved by `ulps` units in its
    last place (away from zero for ulps > 0); returns (planes, exact change)."""
    out = [p.copy() for p in planes]
    x = out[limb][idx]
    step = math.ulp(x) if x != 0 else math.ulp(0.0)
    out[limb][idx] = x + math.copysign(step, x if x != 0 else 1.0) * ulps
    return out, F(out[limb][idx]) - F(x)


def wide_dd(rows, cols, seed, span=600):
    """Canonical DD numbers with exponents spread over +-span binades."""
    g = np.random.default_rng(4242 + seed)
    hi = g.uniform(-1, 1, (rows, cols)) * np.exp2(g.integers(-span, span + 1, (rows, cols)))
    lo = hi * 2.0 ** -53 * g.uniform(-1, 1, (rows, cols))
    s = hi + lo
    return (s, lo - (s - hi))


# --------------------------------------------------------------------------
# cref.exact_diff
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["dd", "qd", "dd_wide", "dd_vs_qd", "qd_vs_fp64"])
def test_exact_diff_matches_fractions(oracle, kind):
    """Independent X and Y, and Y equal to X but for its lower limbs (all the
    leading bits cancel): every element equals the nearest double to the
    exact difference."""
    shape = (7, 9)
    if kind == "dd":
        X, Y = inputs.dd_illcond(*shape, 20), inputs.dd_illcond(*shape, 21)
    elif kind == "qd":
        X, Y = inputs.qd_uniform(*shape, 22), inputs.qd_uniform(*shape, 23)
    elif kind == "dd_wide":
        X, Y = wide_dd(*shape, 0), wide_dd(*shape, 1)
    elif kind == "dd_vs_qd":
        X, Y = inputs.dd_uniform(*shape, 24), inputs.qd_uniform(*shape, 25)
    else:
        X, Y = inputs.qd_uniform(*shape, 26), (inputs.dd_uniform(*shape, 27)[0],)
    # half of the rows: Y shares X's leading limb (cancellation down to the
    # lower limbs); the rest independent
    Y = [y.copy() for y in Y]
    Y[0][::2] = X[0][::2]
    d = oracle.exact_diff(X, Y)
    for idx in np.ndindex(shape):
        assert d[idx] == nearest(value(X, idx) - value(Y, idx)), (kind, idx)


@pytest.mark.parametrize("L", [2, 4])
def test_exact_diff_reports_one_ulp_of_the_last_limb(oracle, L):
    """Y = X exactly gives 0 everywhere; Y = X with the last limb of one entry
    moved by one ulp gives exactly that ulp (with its sign) there and 0
    elsewhere; a checker that ignored the last limb would report 0."""
    X = inputs.dd_uniform(5, 6, 30) if L == 2 else inputs.qd_uniform(5, 6, 31)
    assert not oracle.exact_diff(X, X).any()
    for idx, ulps in (((0, 0), 1), ((3, 4), -1), ((4, 5), 3)):
        Y, delta = nudge(X, L - 1, idx, ulps)
        d = oracle.exact_diff(X, Y)
        assert d[idx] == -float(delta) and d[idx] != 0.0
        mask = np.ones(d.shape, bool)
        mask[idx] = False
        assert not d[mask].any()
        # the same change read with the last limb dropped goes unseen: the
        # pin above is what catches a checker with a dropped term
        assert not oracle.exact_diff(X[:L - 1], Y[:L - 1]).any()


def test_exact_diff_sign_and_ties(oracle):
    """Hand-made cases: the sign of the difference, a difference that is
    exactly halfway between two doubles (ties to even), and a difference
    far below the leading limbs."""
    one = np.array([1.0])
    X = (np.array([1.0, 1.0, 2.0 ** 300]), np.array([2.0 ** -60, 0.0, 2.0 ** 240]))
    Y = (np.array([1.0, 1.0 + 2.0 ** -52, 2.0 ** 300]), np.array([0.0, 0.0, 2.0 ** 240 - 2.0 ** 188]))
    d = oracle.exact_diff(X, Y)
    assert d[0] == 2.0 ** -60
    assert d[1] == -2.0 ** -52
    assert d[2] == 2.0 ** 188
    # 1 + 2^-53 exactly halfway between 1 and 1 + 2^-52: rounds to 1 (even)
    t = oracle.exact_diff((one + 1.0, np.array([2.0 ** -53])), (one,))
    assert t[0] == 1.0
    t = oracle.exact_diff((one + 1.0, np.array([3 * 2.0 ** -53])), (one,))
    assert t[0] == 1.0 + 2.0 ** -51     # 1 + 3 2^-53: nearest is 1 + 2^-51


# --------------------------------------------------------------------------
# exact.entries_exact
# --------------------------------------------------------------------------

def brute_entry(A, B, i, j):
    l = A[0].shape[1]
    c = Fraction(0)
    g = Fraction(0)
    for k in range(l):
        a = value(A, (i, k))
        b = value(B, (k, j))
        c += a * b
        g += abs(a) * abs(b)
    return c, g


@pytest.mark.parametrize("kind", ["dd_illcond", "qd", "fp64_wide"])
def test_entries_exact_matches_brute_force(kind):
    if kind == "dd_illcond":
        A, B = inputs.dd_illcond(6, 11, 40), inputs.dd_illcond(11, 5, 41)
    elif kind == "qd":
        A, B = inputs.qd_uniform(6, 11, 42), inputs.qd_uniform(11, 5, 43)
    else:
        A, B = (inputs.fp64_wide(6, 11, 44),), (inputs.fp64_wide(11, 5, 45),)
    pairs = [(i, j) for i in range(6) for j in range(5)]
    vals, mags = exact.entries_exact(A, B, pairs)
    for (i, j), v, g in zip(pairs, vals, mags):
        c, gg = brute_entry(A, B, i, j)
        assert v == c and g == gg, (kind, i, j)
    # and it agrees with the full exact products
    Ci, s = exact.matmul_exact(A, B)
    Gi, _ = exact.abs_matmul_exact(A, B)
    for (i, j), v, g in zip(pairs, vals, mags):
        assert v == Fraction(int(Ci[i, j]), 2 ** s) and g == Fraction(int(Gi[i, j]), 2 ** s)


def test_entries_exact_sees_a_planted_lower_limb_change():
    """One ulp added to the lo limb of a_23 changes c_2j by exactly that ulp
    times b_3j and leaves the other rows alone; entries out of order and
    repeated rows/columns are handled."""
    A, B = inputs.dd_uniform(5, 7, 46), inputs.dd_uniform(7, 4, 47)
    A2, delta = nudge(A, 1, (2, 3))
    pairs = [(4, 3), (2, 0), (2, 3), (0, 1), (2, 0)]
    v1, _ = exact.entries_exact(A, B, pairs)
    v2, _ = exact.entries_exact(A2, B, pairs)
    for (i, j), x, y in zip(pairs, v1, v2):
        if i == 2:
            assert y - x == delta * value(B, (3, j)) and y != x
        else:
            assert y == x


# --------------------------------------------------------------------------
# exact.error_ratios and the helpers built on it
# --------------------------------------------------------------------------

def test_error_ratios_hand_computed():
    """C = AB rounded to DD, then known errors planted; the ratio must be
    |err| / (l 2^-104 (|A||B|)_ij) exactly (rounded once), 0 for an exact
    entry with (|A||B|)_ij = 0 and inf for an inexact one."""
    A = (np.array([[1.0, 2.0 ** -30, -3.0], [0.0, 0.0, 0.0], [0.5, 0.25, 0.125]]),
         np.array([[2.0 ** -60, 0.0, 2.0 ** -55], [0.0, 0.0, 0.0], [0.0, 2.0 ** -57, 0.0]]))
    B = (np.array([[1.5, -2.0], [7.0, 0.75], [1.0, 1.0]]),
         np.array([[0.0, 2.0 ** -58], [2.0 ** -52, 0.0], [0.0, 0.0]]))
    l = 3
    Ci, s = exact.matmul_exact(A, B)
    Gi, _ = exact.abs_matmul_exact(A, B)
    ex = [[brute_entry(A, B, i, j) for j in range(2)] for i in range(3)]
    C = [np.zeros((3, 2)), np.zeros((3, 2))]
    for i in range(3):
        for j in range(2):
            C[0][i, j], C[1][i, j] = exact.round_to_limbs(ex[i][j][0], 2)
    r0 = exact.error_ratios(C, Ci, s, Gi, l, -104)
    for i in range(3):
        for j in range(2):
            err = abs(value(C, (i, j)) - ex[i][j][0])
            want = 0.0 if ex[i][j][1] == 0 else float(err / (l * ex[i][j][1] * Fraction(2) ** -104))
            assert r0[i, j] == want
    # planted errors: 5 ulps of the lo limb at (0, 1), 1 ulp of hi at (2, 0)
    # and a nonzero value where (|A||B|) = 0 (row 1)
    C2, d1 = nudge(C, 1, (0, 1), 5)
    C2, d2 = nudge(C2, 0, (2, 0), 1)
    C2[0][1, 1] = 2.0 ** -900
    r = exact.error_ratios(C2, Ci, s, Gi, l, -104)
    base = abs(value(C, (0, 1)) - ex[0][1][0])
    want01 = float(abs(value(C2, (0, 1)) - ex[0][1][0]) / (l * ex[0][1][1] * Fraction(2) ** -104))
    assert r[0, 1] == want01 and r[0, 1] > r0[0, 1]
    assert abs(value(C2, (0, 1)) - ex[0][1][0]) <= base + abs(d1)
    want20 = float(abs(value(C2, (2, 0)) - ex[2][0][0]) / (l * ex[2][0][1] * Fraction(2) ** -104))
    assert r[2, 0] == want20 and r[2, 0] > 2.0 ** 40          # an ulp of hi is far out of bound
    assert r[1, 0] == 0.0 and r[1, 1] == math.inf
    # the QD unit divides by 2^-208 instead
    rq = exact.error_ratios(C2, Ci, s, Gi, l, -208)
    assert rq[0, 1] == float(Fraction(want01) * Fraction(2) ** 104) or \
        math.isclose(rq[0, 1], want01 * 2.0 ** 104, rel_tol=2.0 ** -50)


@pytest.mark.parametrize("L,unit", [(2, -104), (4, -208)])
def test_helpers_error_ratio_full_agrees_and_flags(oracle, L, unit):
    """helpers.error_ratio_full (C super-accumulator path, used by every
    full-matrix GPU check) agrees with the Python-integer path, and a
    planted error of twenty times the bound at one entry is reported as
    a ratio above 8 at that entry."""
    m, l, n = 6, 40, 5
    gen = inputs.dd_illcond if L == 2 else inputs.qd_uniform
    A, B = gen(m, l, 50), gen(l, n, 51)
    Cf = oracle.gemm_simple(A, B)
    rf, _ = helpers.error_ratio_full(Cf, A, B, unit)
    rp = helpers.error_ratio_exact_python(Cf, A, B, unit)
    assert rf <= 8 and rp <= 8
    # the C path rounds the error and |A||B| once each and adds a slack for
    # the rounded exact product: it bounds the exact ratio from above, by a
    # margin of a few units of 2^-(53 L) relative to |AB|
    assert rf >= rp * (1 - 2.0 ** -40)
    G = oracle.absprod_exact(A, B)
    C2 = [c.copy() for c in Cf]
    planted = 20 * l * 2.0 ** unit * G[3, 2]
    C2[L - 1][3, 2] += planted
    rf2, r_all = helpers.error_ratio_full(C2, A, B, unit)
    assert rf2 > 8 and r_all[3, 2] > 8
    assert helpers.error_ratio_exact_python(C2, A, B, unit) > 8


def test_helpers_normwise_and_sampled(oracle):
    """normwise_ratio and sampled_errors against Fractions, with a planted
    error."""
    m, l, n = 5, 17, 4
    A, B = inputs.dd_uniform(m, l, 52), inputs.dd_uniform(l, n, 53)
    C = list(oracle.gemm_simple(A, B))
    C, delta = nudge(C, 1, (1, 2), 7)
    exact_err = [[abs(value(C, (i, j)) - brute_entry(A, B, i, j)[0]) for j in range(n)]
                 for i in range(m)]
    amax = max(abs(F(x)) for x in A[0].ravel())
    bmax = max(abs(F(x)) for x in B[0].ravel())
    true_norm = max(max(r) for r in exact_err) / (amax * bmax)
    got = helpers.normwise_ratio(C, A, B, 2)
    # helpers add a slack of one rounding of the exact product and scale the
    # maxima up by 2^-50: within that of the exact value, and never below it
    assert got >= float(true_norm) * (1 - 2.0 ** -45)
    assert got <= float(true_norm) * (1 + 2.0 ** -45) + 2.0 ** -100 * float(
        max(abs(brute_entry(A, B, i, j)[0]) for i in range(m) for j in range(n)) / (amax * bmax))
    pairs = [(1, 2), (0, 0), (4, 3)]
    errs, mags = helpers.sampled_errors(C, A, B, pairs)
    for (i, j), e, g in zip(pairs, errs, mags):
        c, gg = brute_entry(A, B, i, j)
        assert e == float(abs(value(C, (i, j)) - c)) and g == float(gg)
    assert errs[0] >= abs(float(delta)) * 0.5


def test_rows_cols_random_sampler_matches_full_check(oracle):
    """The sampled checker used at full sizes (full rows and columns through
    transposed slabs, random entries one by one) gives, entry for entry, the
    ratios of the full check, and reports a planted one-ulp change of a lower
    limb in a checked row and in a checked column."""
    import numpy as np
    from paper_1710_01839_amd import inputs
    from tests.helpers import rows_cols_random_errors, rows_cols_random_ratios
    from fractions import Fraction
    from oracle import exact
    A, B = inputs.dd_illcond(40, 31, 3), inputs.dd_illcond(31, 27, 4)
    C = oracle.gemm_simple(A, B)
    I, J, err, G = rows_cols_random_errors(C, A, B, nrand=50, seed=3)
    pairs = list(zip(I.tolist(), J.tolist()))
    vals, mags = exact.entries_exact(A, B, pairs)
    for (i, j), v, mg, e, g in zip(pairs, vals, mags, err, G):
        d = abs(exact.limbs_fraction(C, (i, j)) - v)        # the exact error
        assert Fraction(e) >= d and Fraction(e) <= d * (1 + Fraction(1, 2 ** 50)) + abs(v) * Fraction(1, 2 ** 150)
        assert abs(Fraction(g) - mg) <= mg * Fraction(1, 2 ** 52)
    assert set(zip(I[:27].tolist(), J[:27].tolist())) == {(0, j) for j in range(27)}
    I0, J0, err0, _ = rows_cols_random_errors(C, A, B, nrand=0)
    for (i, j) in ((39, 11), (17, 26)):         # last row, last column
        P = (C[0].copy(), C[1].copy())
        P[1][i, j] = np.nextafter(P[1][i, j], np.inf)
        I1, J1, err1, _ = rows_cols_random_errors(P, A, B, nrand=0)
        at = (I0 == i) & (J0 == j)
        assert at.any() and np.all(err1[at] != err0[at]) and np.all(err1[~at] == err0[~at])
    assert rows_cols_random_ratios(C, A, B, -104, nrand=0)[0] <= 8.0
