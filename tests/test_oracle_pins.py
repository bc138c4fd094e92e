"""Pins of the CPU oracle against things other than itself: exact rational
arithmetic, closed forms, integer special cases, brute force on tiny inputs
and the numbers printed in the paper."""
from __future__ import annotations

import csv
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import exact, predict
from paper_1710_01839_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
finite = st.floats(min_value=-2.0 ** 400, max_value=2.0 ** 400, allow_nan=False,
                   allow_infinity=False, allow_subnormal=False)


def F(x) -> Fraction:
    return Fraction(float(x))


def limbs(x) -> Fraction:
    return sum((F(v) for v in x), Fraction(0))


# --------------------------------------------------------------------------
# error-free transforms: the sums and products must be exact identities
# --------------------------------------------------------------------------

@settings(max_examples=300, deadline=None)
@given(finite, finite)
def test_two_sum_exact(oracle, a, b):
    s, e = oracle.two_sum(np.array([a]), np.array([b]))
    assert F(s[0]) + F(e[0]) == F(a) + F(b)
    assert s[0] == a + b                      # s is the rounded sum
    if s[0] != 0:
        assert abs(F(e[0])) <= Fraction(math.ulp(s[0])) / 2


@settings(max_examples=300, deadline=None)
@given(finite, finite)
def test_fast_two_sum_exact_when_ordered(oracle, a, b):
    if abs(a) < abs(b):
        a, b = b, a
    s, e = oracle.fast_two_sum(np.array([a]), np.array([b]))
    assert F(s[0]) + F(e[0]) == F(a) + F(b)


small = st.floats(min_value=-2.0 ** 450, max_value=2.0 ** 450, allow_nan=False,
                  allow_infinity=False, allow_subnormal=False).filter(
    lambda x: x == 0 or abs(x) > 2.0 ** -450)


@settings(max_examples=300, deadline=None)
@given(small, small)
def test_two_prod_exact_and_fma_agrees(oracle, a, b):
    p, e = oracle.two_prod(np.array([a]), np.array([b]), use_fma=False)
    assert F(p[0]) + F(e[0]) == F(a) * F(b)
    p2, e2 = oracle.two_prod(np.array([a]), np.array([b]), use_fma=True)
    assert p2[0] == p[0] and e2[0] == e[0]


def test_two_sum_catches_planted_mistake(oracle):
    """A TwoSum that drops its error term fails the exactness pin."""
    a, b = np.array([1.0]), np.array([2.0 ** -60])
    s, e = oracle.two_sum(a, b)
    assert F(s[0]) + F(e[0]) == F(1.0) + F(2.0 ** -60)
    assert F(s[0]) + 0 != F(1.0) + F(2.0 ** -60)


# --------------------------------------------------------------------------
# DD and QD single operations: error relative to the exact result
# --------------------------------------------------------------------------

def _rand_multi(g, n, L, spread=0):
    x0 = g.uniform(-1, 1, n) * 2.0 ** g.integers(-spread, spread + 1, n)
    out = [x0]
    for _ in range(L - 1):
        _, E = np.frexp(out[-1])
        out.append(np.ldexp(g.uniform(-1, 1, n), E - 54))
    return tuple(out)


@pytest.mark.parametrize("L,unit", [(2, Fraction(1, 2 ** 104)), (4, Fraction(1, 2 ** 208))])
def test_number_ops_error(oracle, L, unit):
    g = np.random.default_rng(1)
    n = 400
    x = _rand_multi(g, n, L, 20)
    y = _rand_multi(g, n, L, 20)
    # adversarial: y close to -x in the leading limbs (heavy cancellation)
    y = tuple(np.where(np.arange(n) % 4 == 0, -xv, yv) for xv, yv in zip(x, y))
    y = (y[0],) + tuple(np.where(np.arange(n) % 4 == 0, yv * 0.5, yv) for yv in y[1:])
    s = oracle.num_op("add", x, y)
    p = oracle.num_op("mul", x, y)
    for i in range(n):
        xi = limbs(v[i] for v in x)
        yi = limbs(v[i] for v in y)
        si = limbs(v[i] for v in s)
        pi = limbs(v[i] for v in p)
        assert abs(si - (xi + yi)) <= 4 * unit * (abs(xi) + abs(yi))
        assert abs(pi - xi * yi) <= 8 * unit * abs(xi * yi)


# --------------------------------------------------------------------------
# exact products
# --------------------------------------------------------------------------

def _brute_force(A, B):
    m, l = A[0].shape
    n = B[0].shape[1]
    return [[sum(limbs(p[i, k] for p in A) * limbs(q[k, j] for q in B) for k in range(l))
             for j in range(n)] for i in range(m)]


def test_python_exact_matches_brute_force():
    A = inputs.dd_illcond(5, 7, 0)
    B = inputs.dd_illcond(7, 4, 1)
    Ci, s = exact.matmul_exact(A, B)
    bf = _brute_force(A, B)
    for i in range(5):
        for j in range(4):
            assert Fraction(int(Ci[i, j]), 2 ** s) == bf[i][j]


def test_closed_form_of_paper_sum():
    """sum_k (i + k - 1)(n - k) = n(n - 1)(3i + n - 2)/6 (k = 1..n), the
    integer identity behind the paper's test matrices; checked by brute
    force and through the exact GEMM on the integer parts."""
    for n in range(1, 12):
        for i in range(1, n + 1):
            assert sum((i + k - 1) * (n - k) for k in range(1, n + 1)) * 6 == \
                n * (n - 1) * (3 * i + n - 2)
    n = 9
    A = (np.add.outer(np.arange(1, n + 1), np.arange(1, n + 1)).astype(float) - 1.0,)
    B = (np.repeat((n - np.arange(1, n + 1))[:, None], n, axis=1).astype(float),)
    Ci, s = exact.matmul_exact(A, B)
    for i in range(1, n + 1):
        for j in range(n):
            assert int(Ci[i - 1, j]) * 6 == n * (n - 1) * (3 * i + n - 2) * 2 ** s


def test_paper_matrices_are_nearest_multilimb():
    """Each entry of A = [sqrt5 (i+j-1)] is within 2^-210 relative of the real value."""
    A, B = inputs.paper_matrices(6, 4)
    for (i, j) in ((0, 0), (2, 3), (5, 5)):
        v = i + j + 1
        x = limbs(p[i, j] for p in A)
        assert abs(x * x - 5 * v * v) <= Fraction(5 * v * v, 2 ** 205)
    x = limbs(p[0, 0] for p in B)     # sqrt3 (n - 1)
    assert abs(x * x - 3 * 25) <= Fraction(75, 2 ** 205)


@pytest.mark.parametrize("kind", ["dd", "qd", "illcond", "fp64"])
def test_c_exact_equals_python_exact(oracle, kind):
    """The super-accumulator product, rounded limb by limb to nearest, equals
    the Python-integer product rounded the same way, bit for bit."""
    if kind == "dd":
        A, B = inputs.dd_uniform(9, 13, 2), inputs.dd_uniform(13, 6, 3)
    elif kind == "qd":
        A, B = inputs.qd_uniform(7, 11, 4), inputs.qd_uniform(11, 5, 5)
    elif kind == "illcond":
        A, B = inputs.dd_illcond(8, 40, 6), inputs.dd_illcond(40, 7, 7)
    else:
        A, B = (inputs.fp64_wide(6, 30, 8),), (inputs.fp64_wide(30, 5, 9),)
    L = max(len(A), 2)
    Ce = oracle.gemm_exact(A, B, out_limbs=L)
    Ci, s = exact.matmul_exact(A, B)
    for i in range(Ce[0].shape[0]):
        for j in range(Ce[0].shape[1]):
            want = exact.round_to_limbs(Fraction(int(Ci[i, j]), 2 ** s), L)
            assert [Ce[q][i, j] for q in range(L)] == want


def test_absprod_exact(oracle):
    A, B = inputs.dd_illcond(6, 25, 10), inputs.dd_illcond(25, 4, 11)
    G = oracle.absprod_exact(A, B)
    Gi, s = exact.abs_matmul_exact(A, B)
    for i in range(6):
        for j in range(4):
            assert G[i, j] == exact.round_to_limbs(Fraction(int(Gi[i, j]), 2 ** s), 1)[0]


# --------------------------------------------------------------------------
# step-by-step DD / QD simple GEMM and Strassen
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L,gen", [(2, inputs.dd_uniform), (2, inputs.dd_illcond),
                                   (4, inputs.qd_uniform)])
def test_simple_gemm_within_bound(oracle, L, gen):
    m, l, n = 12, 64, 9
    A, B = gen(m, l, 12), gen(l, n, 13)
    C = oracle.gemm_simple(A, B)
    Ci, s = exact.matmul_exact(A, B)
    Gi, _ = exact.abs_matmul_exact(A, B)
    r = exact.error_ratios(C, Ci, s, Gi, l, -104 if L == 2 else -208)
    assert r.max() <= 8.0


@pytest.mark.parametrize("L,bits", [(2, 30), (4, 60)])
def test_integer_inputs_exact(oracle, L, bits):
    """Integer inputs: every step is exact, so the simple GEMM and both
    Strassen forms give exactly AB (canonical limbs)."""
    m, l, n = 10, 48, 12
    A, B = inputs.integers(m, l, L, 14, bits), inputs.integers(l, n, L, 15, bits)
    want = oracle.gemm_exact(A, B, out_limbs=L)
    got = [oracle.gemm_simple(A, B)]
    for d in (1, 2):
        got.append(oracle.gemm_strassen(A, B, d, "classic"))
        got.append(oracle.gemm_strassen(A, B, d, "winograd"))
    for C in got:
        for q in range(L):
            assert np.array_equal(C[q], want[q])


def test_strassen_rectangular_and_odd_integer(oracle):
    """Eq. (3) holds for rectangular even blocks; odd sizes are zero-padded."""
    A, B = inputs.integers(7, 13, 2, 16, 20), inputs.integers(13, 5, 2, 17, 20)
    want = oracle.gemm_exact(A, B, out_limbs=2)
    for v in ("classic", "winograd"):
        for d in (1, 2, 3):
            C = oracle.gemm_strassen(A, B, d, v)
            assert np.array_equal(C[0], want[0]) and np.array_equal(C[1], want[1])


@pytest.mark.parametrize("L", [2, 4])
def test_strassen_normwise_bound(oracle, L):
    from tests.helpers import classic_bound, normwise_ratio, winograd_bound
    n = 64
    gen = inputs.dd_uniform if L == 2 else inputs.qd_uniform
    A, B = gen(n, n, 18), gen(n, n, 19)
    unit = 8 * 2.0 ** (-104 if L == 2 else -208)
    for d in (1, 2):
        r = normwise_ratio(oracle.gemm_strassen(A, B, d, "classic"), A, B, L)
        assert r <= classic_bound(n, d, unit)
        r = normwise_ratio(oracle.gemm_strassen(A, B, d, "winograd"), A, B, L)
        assert r <= winograd_bound(n, d, unit)


# --------------------------------------------------------------------------
# the prediction rule against the paper's Tables 1 and 3
# --------------------------------------------------------------------------

def _rows():
    with open(os.path.join(HERE, "golden", "prediction_tables.csv")) as f:
        return list(csv.DictReader(line for line in f if not line.startswith("#")))


def _half_unit(s: str) -> float:
    return 0.5 * 10.0 ** -(len(s.split(".")[1]) if "." in s else 0)


def test_prediction_rule_reproduces_tables():
    rows = _rows()
    assert len(rows) == 44
    n = 1024
    for r in rows:
        nm = int(r["n_min"])
        c, d, b = float(r["predict_cost_c"]), float(r["predicted_d"]), float(r["real_b"])
        pred = predict.predict_full_time(c, n, nm)
        tol = _half_unit(r["predict_cost_c"]) * n / predict.slab_rows(n, nm) + _half_unit(r["predicted_d"])
        assert abs(pred - d) <= tol + 1e-12, r
        rd = 100 * predict.rel_diff(d, b)
        assert abs(rd - float(r["rel_diff_pct"])) <= 0.0051 + 100 * _half_unit(r["predicted_d"]) / b, r


def test_prediction_rule_rejects_other_readings():
    """Slabs of n_min rows, or quadratic scaling, do not reproduce the tables."""
    rows = _rows()
    bad1 = sum(abs(float(r["predict_cost_c"]) * 1024 / int(r["n_min"]) - float(r["predicted_d"]))
               > 0.02 * float(r["predicted_d"]) for r in rows)
    bad2 = sum(abs(float(r["predict_cost_c"]) * (1024 / (2 * int(r["n_min"]))) ** 2
                   - float(r["predicted_d"])) > 0.02 * float(r["predicted_d"]) for r in rows
               if 2 * int(r["n_min"]) < 1024)
    assert bad1 >= 40 and bad2 >= 30


def test_tuning_procedure_three_steps():
    """Steps (1)-(3): slab predictions for every candidate, then exactly three
    full-size timings, fastest wins."""
    costs = {8: 9.0, 16: 5.0, 32: 4.0, 64: 4.5}

    def slab(nm, rows):
        return costs[nm] * rows / 1024

    def full(algo, nm):
        return {"simple": 10.0, "block": costs[nm], "strassen": 3.5}[algo]

    algo, nm, log = predict.tune(1024, [8, 16, 32, 64], slab, full)
    assert nm == 32 and algo == "strassen"
    assert [k for k, _, _ in log] == ["slab"] * 4 + ["simple", "block", "strassen"]
