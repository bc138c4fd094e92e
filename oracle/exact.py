"""Exact oracle in Python integers: C = AB of Eq. (1) with no rounding.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

Every double is a dyadic rational M * 2^E with an integer M, so a matrix of
multi-limb numbers (limb planes) is turned into integers on one common scale
and multiplied with Python's unbounded integers.  Nothing here rounds, so this
is the definition of the product the paper's methods approximate.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def _mant_exp(x: np.ndarray):
    """x == M * 2^E elementwise, M an int64 with |M| < 2^53 (0 for x == 0)."""
    fr, e = np.frexp(np.asarray(x, dtype=np.float64))
    M = np.ldexp(fr, 53).astype(np.int64)
    E = e.astype(np.int64) - 53
    return M, E


def scale_of(planes) -> int:
    """Smallest s such that every limb times 2^s is an integer (s >= 0)."""
    s = 0
    for p in planes:
        M, E = _mant_exp(p)
        nz = M != 0
        if nz.any():
            s = max(s, int(-E[nz].min()))
    return s


def to_int(planes, s: int) -> np.ndarray:
    """Object array of Python ints equal to (sum of limbs) * 2^s exactly."""
    out = None
    for p in planes:
        M, E = _mant_exp(p)
        sh = E + s
        if (sh[M != 0] < 0).any():
            raise ValueError("scale too small for an exact integer image")
        sh = np.where(M != 0, sh, 0)
        Mo = M.astype(object)
        term = np.vectorize(lambda m, k: int(m) << int(k), otypes=[object])(Mo, sh)
        out = term if out is None else out + term
    return out


def matmul_exact(A, B):
    """Exact AB for limb-plane matrices.  Returns (C_int, sA + sB): the object
    array of integers and the power of two they are scaled by."""
    sA, sB = scale_of(A), scale_of(B)
    Ai, Bi = to_int(A, sA), to_int(B, sB)
    return Ai.dot(Bi), sA + sB


def abs_matmul_exact(A, B):
    sA, sB = scale_of(A), scale_of(B)
    Ai, Bi = to_int(A, sA), to_int(B, sB)
    f = np.vectorize(abs, otypes=[object])
    return f(Ai).dot(f(Bi)), sA + sB


def entries_exact(A, B, pairs):
    """Exact c_ij and (|A||B|)_ij for selected (i, j) only (large matrices).
    Returns lists of Fractions."""
    rows = sorted({i for i, _ in pairs})
    cols = sorted({j for _, j in pairs})
    Ar = [np.ascontiguousarray(p[rows, :]) for p in A]
    Bc = [np.ascontiguousarray(p[:, cols]) for p in B]
    sA, sB = scale_of(Ar), scale_of(Bc)
    Ai, Bi = to_int(Ar, sA), to_int(Bc, sB)
    ri = {r: t for t, r in enumerate(rows)}
    ci = {c: t for t, c in enumerate(cols)}
    den = 1 << (sA + sB)
    vals, mags = [], []
    for i, j in pairs:
        a = Ai[ri[i], :]
        b = Bi[:, ci[j]]
        c = sum(int(x) * int(y) for x, y in zip(a, b))
        g = sum(abs(int(x)) * abs(int(y)) for x, y in zip(a, b))
        vals.append(Fraction(c, den))
        mags.append(Fraction(g, den))
    return vals, mags


def limbs_fraction(planes, idx) -> Fraction:
    """Exact value of the multi-limb number at index idx."""
    return sum((Fraction(float(p[idx])) for p in planes), Fraction(0))


def error_ratios(C, C_int, s: int, absAB_int, l: int, unit_exp: int):
    """Componentwise ratio |C - exact|_ij / (l * 2^unit_exp * (|A||B|)_ij),
    computed exactly and returned as float64.  unit_exp is -104 for the DD
    bound and -208 for the QD bound.  Entries with (|A||B|)_ij == 0 must be
    exact and get ratio 0 (or inf when they are not)."""
    sC = max(s, scale_of(C))
    Cg = to_int(C, sC)
    up = 1 << (sC - s)
    out = np.zeros(C[0].shape)
    it = np.ndindex(C[0].shape)
    for idx in it:
        err = abs(int(Cg[idx]) - int(C_int[idx]) * up)
        mag = int(absAB_int[idx]) * up
        if mag == 0:
            out[idx] = 0.0 if err == 0 else math.inf
        else:
            # err / (l * 2^unit_exp * mag)
            out[idx] = float(Fraction(err, l * mag) / Fraction(2) ** unit_exp)
    return out


def round_to_limbs(value: Fraction, limbs: int):
    """Round-to-nearest limb extraction of an exact rational."""
    out = []
    r = value
    for _ in range(limbs):
        d = _fraction_to_double(r)
        out.append(d)
        r = r - Fraction(d)
    return out


def _fraction_to_double(r: Fraction) -> float:
    # int / int true division in Python is correctly rounded.
    return r.numerator / r.denominator if r != 0 else 0.0
