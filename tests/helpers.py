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


class ExactSample:
    """The exact AB and (|A||B|) on full rows, full columns (default: the
    first and last of each) and `nrand` random entries, from the oracle's
    exact super-accumulator, computed once for checking several results.
    Row slabs are computed as (B^T A_rows^T)^T, which has the same exact
    terms, so the oracle runs in parallel over B's columns.  Flat arrays:
    I, J (entry indices), Ce (limb tuple of AB rounded limb by limb, 3
    limbs), G ((|A||B|)_ij rounded to nearest)."""

    def __init__(self, A, B, rows=None, cols=None, nrand: int = 1024, seed: int = 7, threads: int = 0):
        m, l = A[0].shape
        n = B[0].shape[1]
        self.l = l
        rows = [0, m - 1] if rows is None else list(rows)
        cols = [0, n - 1] if cols is None else list(cols)
        I, J, Ce, G = [], [], [], []

        def add(ii, jj, ce, g):
            I.append(np.broadcast_to(ii, g.shape).ravel())
            J.append(np.broadcast_to(jj, g.shape).ravel())
            Ce.append([x.ravel() for x in ce])
            G.append(np.asarray(g).ravel())

        BT = tuple(np.ascontiguousarray(p.T) for p in B)
        Ar = tuple(np.ascontiguousarray(p[rows].T) for p in A)
        add(np.array(rows)[:, None], np.arange(n)[None, :],
            tuple(np.ascontiguousarray(x.T) for x in cref.gemm_exact(BT, Ar, out_limbs=3, threads=threads)),
            np.ascontiguousarray(cref.absprod_exact(BT, Ar, threads=threads).T))
        del BT
        Bc = tuple(np.ascontiguousarray(p[:, cols]) for p in B)
        add(np.arange(m)[:, None], np.array(cols)[None, :], cref.gemm_exact(A, Bc, out_limbs=3, threads=threads),
            cref.absprod_exact(A, Bc, threads=threads))
        g = np.random.default_rng(seed)
        for _ in range(nrand):
            i, j = int(g.integers(0, m)), int(g.integers(0, n))
            Ai = tuple(np.ascontiguousarray(p[i:i + 1]) for p in A)
            Bj = tuple(np.ascontiguousarray(p[:, j:j + 1]) for p in B)
            add(np.array([[i]]), np.array([[j]]), cref.gemm_exact(Ai, Bj, out_limbs=3, threads=1),
                cref.absprod_exact(Ai, Bj, threads=1))
        self.I, self.J = np.concatenate(I), np.concatenate(J)
        self.Ce = tuple(np.concatenate([c[q] for c in Ce]) for q in range(3))
        self.G = np.concatenate(G)

    def errors(self, C):
        """|C - AB| at the sampled entries: the difference from the 3-limb
        rounding of AB rounded once, plus the slack of both roundings."""
        Cs = tuple(np.ascontiguousarray(c[self.I, self.J]) for c in C)
        d = np.abs(cref.exact_diff(Cs, self.Ce))
        return d + np.abs(self.Ce[0]) * 2.0 ** -160 + d * 2.0 ** -52

    def ratios(self, C, unit_exp: int):
        """|C - AB|_ij / (l 2^unit_exp (|A||B|)_ij) at the sampled entries."""
        err = self.errors(C)
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(self.G > 0, err / (self.l * 2.0 ** unit_exp * self.G),
                            np.where(err > 0, np.inf, 0.0))


def rows_cols_random_errors(C, A, B, rows=None, cols=None, nrand: int = 1024, seed: int = 7,
                            threads: int = 0):
    """(I, J, |C - AB|, (|A||B|)) at the entries of ExactSample(A, B, ...)."""
    s = ExactSample(A, B, rows, cols, nrand, seed, threads)
    return s.I, s.J, s.errors(C), s.G


def rows_cols_random_ratios(C, A, B, unit_exp: int, rows=None, cols=None, nrand: int = 1024,
                            seed: int = 7, threads: int = 0):
    """max over the entries of rows_cols_random_errors of
    |C - AB|_ij / (l 2^unit_exp (|A||B|)_ij), and the max error."""
    l = A[0].shape[1]
    _, _, err, G = rows_cols_random_errors(C, A, B, rows, cols, nrand, seed, threads)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(G > 0, err / (l * 2.0 ** unit_exp * G), np.where(err > 0, np.inf, 0.0))
    return float(r.max()), float(err.max())
