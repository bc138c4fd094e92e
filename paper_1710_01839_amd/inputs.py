"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws and lays out numbers (numpy random draws, exact
power-of-two scaling with ldexp, integer square roots); it holds none of the
multiple-precision arithmetic of the method.  Matrices of multi-limb numbers
are tuples of C-contiguous float64 limb planes, leading limb first.

Recipes (the distributions of the paper's workloads and of the synthetic
configurations built around them):

* ``dd_uniform``: hi ~ U[-1, 1]; lo uniform inside hi's canonical half-ulp
  (|lo| < ulp(hi)/2, the scale of hi * 2^-53 * u).
* ``dd_illcond``: the same with hi scaled by 2^k, k ~ U{-30..30} per element.
* ``qd_uniform``: limb 0 ~ U[-1, 1]; limb k uniform inside limb k-1's
  half-ulp, so the four limbs never overlap.
* ``fp64_wide``: plain doubles U[-1, 1] * 2^e with e = round(N(0, 10)) per
  element (inputs of the split-precision integer path).
* ``integers``: integer-valued doubles in [-2^bits, 2^bits], lower limbs 0.
* ``paper_matrices``: A = [sqrt(5)(i + j - 1)], B = [sqrt(3)(n - i)] of the
  paper's experiments, each entry the multi-limb number nearest to the real
  value (computed with integer square roots).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

SEED_BASE = 1710_01839


def rng(seed_offset: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + seed_offset)


def _half_ulp_exponent(x: np.ndarray) -> np.ndarray:
    # x = fr * 2^E with 0.5 <= |fr| < 1, so ulp(x) = 2^(E-53), half-ulp 2^(E-54)
    _, E = np.frexp(x)
    return E - 54


def _next_limb(g: np.random.Generator, prev: np.ndarray) -> np.ndarray:
    u = g.uniform(-1.0, 1.0, size=prev.shape)
    out = np.ldexp(u, _half_ulp_exponent(prev))
    return np.where(prev == 0.0, 0.0, out)


def dd_uniform(rows: int, cols: int, seed_offset: int = 0):
    g = rng(seed_offset)
    hi = g.uniform(-1.0, 1.0, size=(rows, cols))
    lo = _next_limb(g, hi)
    return (np.ascontiguousarray(hi), np.ascontiguousarray(lo))


def dd_illcond(rows: int, cols: int, seed_offset: int = 0, kmax: int = 30):
    g = rng(seed_offset)
    hi = g.uniform(-1.0, 1.0, size=(rows, cols))
    k = g.integers(-kmax, kmax + 1, size=(rows, cols))
    hi = np.ldexp(hi, k)
    lo = _next_limb(g, hi)
    return (np.ascontiguousarray(hi), np.ascontiguousarray(lo))


def qd_uniform(rows: int, cols: int, seed_offset: int = 0, illcond: bool = False):
    g = rng(seed_offset)
    x0 = g.uniform(-1.0, 1.0, size=(rows, cols))
    if illcond:
        x0 = np.ldexp(x0, g.integers(-30, 31, size=(rows, cols)))
    limbs = [x0]
    for _ in range(3):
        limbs.append(_next_limb(g, limbs[-1]))
    return tuple(np.ascontiguousarray(x) for x in limbs)


def fp64_wide(rows: int, cols: int, seed_offset: int = 0, sigma: float = 10.0):
    g = rng(seed_offset)
    u = g.uniform(-1.0, 1.0, size=(rows, cols))
    e = np.rint(g.normal(0.0, sigma, size=(rows, cols))).astype(np.int64)
    return np.ascontiguousarray(np.ldexp(u, e))


def integers(rows: int, cols: int, limbs: int, seed_offset: int = 0, bits: int = 30):
    g = rng(seed_offset)
    hi = g.integers(-(1 << bits), (1 << bits) + 1, size=(rows, cols)).astype(np.float64)
    return tuple([np.ascontiguousarray(hi)] + [np.zeros((rows, cols)) for _ in range(limbs - 1)])


def with_limbs(planes, limbs: int):
    """Pad (with zero planes) or check a limb-plane tuple to ``limbs`` limbs."""
    planes = tuple(planes)
    if len(planes) >= limbs:
        return planes[:limbs]
    z = np.zeros_like(planes[0])
    return planes + tuple(z.copy() for _ in range(limbs - len(planes)))


def _nearest_limbs_of_sqrt(c: int, v: int, limbs: int, bits: int = 480):
    """Limbs of v * sqrt(c) (v >= 0): floor(v sqrt(c) 2^bits) by integer
    square root, then limb-by-limb nearest doubles (int/int true division in
    Python is correctly rounded)."""
    N = math.isqrt(c * v * v << (2 * bits))
    r = Fraction(N, 1 << bits)
    out = []
    for _ in range(limbs):
        d = r.numerator / r.denominator if r != 0 else 0.0
        out.append(d)
        r -= Fraction(d)
    return out


def paper_matrices(n: int, limbs: int):
    """A = [sqrt(5)(i + j - 1)], B = [sqrt(3)(n - i)], i, j = 1..n."""
    vals_a = {v: _nearest_limbs_of_sqrt(5, v, limbs) for v in range(1, 2 * n)}
    vals_b = {v: _nearest_limbs_of_sqrt(3, v, limbs) for v in range(0, n)}
    ia = np.add.outer(np.arange(1, n + 1), np.arange(1, n + 1)) - 1   # i + j - 1
    ib = np.repeat((n - np.arange(1, n + 1))[:, None], n, axis=1)      # n - i
    A, B = [], []
    for q in range(limbs):
        ta = np.array([vals_a[v][q] for v in range(1, 2 * n)])
        tb = np.array([vals_b[v][q] for v in range(0, n)])
        A.append(np.ascontiguousarray(ta[ia - 1]))
        B.append(np.ascontiguousarray(tb[ib]))
    return tuple(A), tuple(B)


def batch_shapes(count: int = 512, lo: int = 16, hi: int = 512, seed_offset: int = 7):
    """(m, n, l) per problem, each log-uniform in [lo, hi]."""
    g = rng(seed_offset)
    x = np.exp(g.uniform(math.log(lo), math.log(hi), size=(count, 3)))
    return [tuple(int(v) for v in row) for row in np.rint(x).astype(np.int64)]


def mlp_init(features: int = 15, hidden: int = 64, seed_offset: int = 11):
    """He-uniform float32 weights, zero biases, for features->hidden->hidden->1."""
    g = rng(seed_offset)

    def u(fan_in, shape):
        lim = math.sqrt(6.0 / fan_in)
        return g.uniform(-lim, lim, size=shape).astype(np.float32)

    return {
        "W1": u(features, (hidden, features)), "b1": np.zeros(hidden, np.float32),
        "W2": u(hidden, (hidden, hidden)), "b2": np.zeros(hidden, np.float32),
        "W3": u(hidden, (1, hidden)), "b3": np.zeros(1, np.float32),
    }
