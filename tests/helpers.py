"""Shared checks for the parity tests (exact error ratios against the oracle)."""
from __future__ import annotations

import numpy as np

from oracle import cref, exact


def error_ratio_full(C, A, B, unit_exp: int, threads: int = 0):
    """max_ij |C - AB|_ij / (l 2^unit_exp (|A||B|)_ij) over all entries, with
    AB and |A||B| from the oracle's exact super-accumulator.  C_exact is the
    limb-by-limb nearest rounding of AB (within 2^-(53 L + 1) |AB| of it);
    the difference C - C_exact is rounded once more to a double.  Both of
    those are added to the error before dividing."""
    L = len(C)
    l = A[0].shape[1]
    Ce = cref.gemm_exact(A, B, out_limbs=L, threads=threads)
    G = cref.absprod_exact(A, B, threads=threads)
    d = np.abs(cref.exact_diff(C, Ce))
    slack = np.abs(Ce[0]) * 2.0 ** (-53 * L - 1) + d * 2.0 ** -52
    err = d + slack
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(G > 0, err / (l * 2.0 ** unit_exp * G), np.where(err > 0, np.inf, 0.0))
    return float(r.max()), r


def error_ratio_exact_python(C, A, B, unit_exp: int):
    """The same ratio computed entirely in Python integers (no rounding)."""
    Ci, s = exact.matmul_exact(A, B)
    Gi, _ = exact.abs_matmul_exact(A, B)
    r = exact.error_ratios(C, Ci, s, Gi, A[0].shape[1], unit_exp)
    return float(r.max())


def sampled_pairs(m: int, n: int, count: int, seed: int = 5):
    g = np.random.default_rng(seed)
    pairs = {(0, 0), (m - 1, n - 1), (0, n - 1), (m - 1, 0)}
    while len(pairs) < count:
        pairs.add((int(g.integers(0, m)), int(g.integers(0, n))))
    return sorted(pairs)


def sampled_errors(C, A, B, pairs):
    """Exact |C - AB|_ij and (|A||B|)_ij at selected entries (as floats,
    computed as Fractions and rounded once at the end)."""
    vals, mags = exact.entries_exact(A, B, pairs)
    errs = []
    for (i, j), v in zip(pairs, vals):
        c = exact.limbs_fraction(C, (i, j))
        errs.append(float(abs(c - v)))
    return errs, [float(g) for g in mags]


def normwise_ratio(C, A, B, limbs_out: int, threads: int = 0):
    """max|C - AB| / (max|A| max|B|), exact error rounded once."""
    Ce = cref.gemm_exact(A, B, out_limbs=limbs_out, threads=threads)
    d = np.abs(cref.exact_diff(C, Ce)) + np.abs(Ce[0]) * 2.0 ** (-53 * limbs_out - 1)
    amax = np.abs(A[0]).max() * (1 + 2.0 ** -50)
    bmax = np.abs(B[0]).max() * (1 + 2.0 ** -50)
    return float(d.max() / (amax * bmax))


def winograd_bound(n: int, depth: int, unit: float) -> float:
    """Normwise bound max|C - C^| <= [18^d (n0^2 + 6 n0) - 6 n] unit max|A| max|B|
    for d levels of Winograd's variant over a conventional product of size
    n0 = n / 2^d with componentwise unit roundoff `unit` (Higham's analysis of
    the Strassen-Winograd recursion, with the DD/QD per-operation error in
    place of the binary64 unit roundoff)."""
    n0 = n / 2 ** depth
    return (18 ** depth * (n0 * n0 + 6 * n0) - 6 * n) * unit


def classic_bound(n: int, depth: int, unit: float) -> float:
    """The same for the classic form of Eq. (3): [12^d (n0^2 + 5 n0) - 5 n]."""
    n0 = n / 2 ** depth
    return (12 ** depth * (n0 * n0 + 5 * n0) - 5 * n) * unit
