"""Split-precision (Ozaki-scheme) product, written out plainly.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

The method (Ozaki, Ogita, Oishi and Rump's error-free splitting, in the
INT8 form of Ootomo, Ozaki and Yokota) reaches double-double accuracy from
products of small integers.  The digits here are radix-256 signed bytes:

1. row scale e_i: the smallest integer with max_k |a_ik| < 2^e_i (0 for a
   zero row); column scale f_j of B likewise;
2. y = a_ik 2^-(e_i + 2) lies in (-1/4, 1/4); digits by truncation toward
   zero, T_1 = trunc(256 y) in [-63, 63], r_1 = 256 y - T_1,
   T_s = trunc(256 r_{s-1}) in [-255, 255], r_s = 256 r_{s-1} - T_s (every
   r_s has the sign of y and |r_s| < 1; each step is exact in binary64), so
   y = sum_s T_s 256^-s + 256^-S r_S;
3. the kept digits are made signed bytes by a carry from the least
   significant up: with c = 0, for s = S .. 2: u = T_s + c,
   c = [u >= 128] - [u < -128], D_s = u - 256 c; D_1 = T_1 + c in [-64, 64].
   The sum of the kept digits is unchanged; every D_s is in [-128, 127];
4. for each kept pair of digit planes (s, t) the integer product
   D_A^(s) D_B^(t) is exact; pairs on one diagonal g = s + t share the
   weight 2^(e_i + f_j + 4 - 8g);
5. C_ij = sum_g 2^(e_i + f_j + 4 - 8g) G_g[i, j].

Every element whose lowest set bit is at or above 2^(e_i + 2 - 8S) is held
exactly by S digits: S = ceil((e_i + 2 - lowest bit) / 8).

Double-double inputs (hi + lo) are split as one exact value (steps 2-3 on
the exact y = (hi + lo) 2^-(e_i + 2)); the scale e_i comes from the hi
limbs.

Pairs kept: all S^2 ('all') or the triangle s + t <= S + 1 ('triangle').
This module forms the digit planes exactly, the diagonal sums with int64
matrix products and the combination exactly in Python integers, then rounds
to double-double (nearest, limb by limb).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from oracle import exact


def row_exponents(A: np.ndarray) -> np.ndarray:
    M = np.abs(A).max(axis=1) if A.shape[1] else np.zeros(A.shape[0])
    _, E = np.frexp(M)              # M = f 2^E with 0.5 <= f < 1, so M < 2^E
    return np.where(M > 0, E, 0).astype(np.int64)


def col_exponents(B: np.ndarray) -> np.ndarray:
    return row_exponents(np.ascontiguousarray(B.T))


def signed_bytes(T):
    """Step 3: truncated digits T (list of int64 arrays, most significant
    first) -> signed-byte digits with the same sum, carrying from the least
    significant digit up."""
    D = [np.array(x, dtype=np.int64) for x in T]
    c = np.zeros_like(D[0]) if D else None
    for s in range(len(D) - 1, 0, -1):
        u = D[s] + c
        c = (u >= 128).astype(np.int64) - (u < -128).astype(np.int64)
        D[s] = u - 256 * c
    if D:
        D[0] = D[0] + c
    return [x.astype(np.int8) for x in D]


def split_rows(X: np.ndarray, e: np.ndarray, S: int):
    """Digit planes (S arrays of int8, same shape as X) of X scaled by
    2^-(e_i + 2) per row, and the scaled remainder r_S (|r_S| < 1, units of
    the last digit, the sign of x).  Multiplying by 256 and removing the
    integer part toward zero are exact in binary64."""
    y = np.ldexp(X, -(e[:, None] + 2))
    T = []
    for _ in range(S):
        v = y * 256.0
        t = np.trunc(v)
        y = v - t
        T.append(t.astype(np.int64))
    return signed_bytes(T), y


def split_cols(X: np.ndarray, f: np.ndarray, S: int):
    d, y = split_rows(np.ascontiguousarray(X.T), f, S)
    return [np.ascontiguousarray(x.T) for x in d], np.ascontiguousarray(y.T)


def split_rows_limbs(X, e: np.ndarray, S: int):
    """Digit planes of the multi-limb values X[0] + X[1] + ... (double-
    double or quad-double) scaled by 2^-(e_i + 2) per row, steps 2-3 in
    exact rational arithmetic (small inputs only).  Returns the planes and
    the exact remainders r_S (object array)."""
    R, K = X[0].shape
    T = [np.zeros((R, K), dtype=np.int64) for _ in range(S)]
    rem = np.empty((R, K), dtype=object)
    for i in range(R):
        scale = Fraction(2) ** int(-(e[i] + 2))
        for k in range(K):
            r = sum(Fraction(float(x[i, k])) for x in X) * scale
            for s in range(S):
                v = 256 * r
                d = int(v)             # toward zero
                T[s][i, k] = d
                r = v - d
            rem[i, k] = r
    return signed_bytes(T), rem


def split_rows_dd(Xhi: np.ndarray, Xlo: np.ndarray, e: np.ndarray, S: int):
    """split_rows_limbs for double-double values hi + lo."""
    return split_rows_limbs((Xhi, Xlo), e, S)


def split_cols_limbs(X, f: np.ndarray, S: int):
    D, rem = split_rows_limbs(tuple(np.ascontiguousarray(x.T) for x in X), f, S)
    return [np.ascontiguousarray(x.T) for x in D], rem.T


def split_cols_dd(Xhi: np.ndarray, Xlo: np.ndarray, f: np.ndarray, S: int):
    return split_cols_limbs((Xhi, Xlo), f, S)


def slices_needed_rows(X: np.ndarray, e: np.ndarray) -> int:
    """Smallest S for which split_rows reproduces every entry exactly:
    ceil((e_i + 2 - exponent of the lowest set bit of x) / 8), maximised."""
    M, E = exact._mant_exp(X)
    nz = M != 0
    if not nz.any():
        return 0
    Mabs = np.abs(M[nz])
    tz = np.zeros(Mabs.shape, dtype=np.int64)
    for b in range(53):
        tz += ((Mabs >> b) & 1 == 0) & (tz == b)
    low = E[nz] + tz                           # x = odd * 2^low
    eb = np.broadcast_to(e[:, None], X.shape)[nz]
    bits = eb + 2 - low
    return int(max(0, np.ceil(bits.max() / 8)))


def slices_exact(A, B) -> int:
    """Slices that make every digit expansion exact.  A, B: FP64 arrays or
    limb tuples (double-double, quad-double); a tuple needs the lowest set
    bit of any limb, against the scale of the leading limbs."""
    Ap = A if isinstance(A, tuple) else (A,)
    Bp = B if isinstance(B, tuple) else (B,)
    e, f = row_exponents(Ap[0]), col_exponents(Bp[0])
    need = [slices_needed_rows(x, e) for x in Ap]
    need += [slices_needed_rows(np.ascontiguousarray(x.T), f) for x in Bp]
    return max(need)


def pairs(S: int, mode: str = "all"):
    """Kept (s, t), 1-based."""
    out = []
    for s in range(1, S + 1):
        for t in range(1, S + 1):
            if mode == "all" or s + t <= S + 1:
                out.append((s, t))
    return out


def group_sums(DA, DB, S: int, mode: str = "all"):
    """{g: sum over kept pairs with s + t = g of D_A^(s) D_B^(t)} (int64)."""
    G = {}
    for s, t in pairs(S, mode):
        P = DA[s - 1].astype(np.int64) @ DB[t - 1].astype(np.int64)
        G[s + t] = G.get(s + t, 0) + P
    return G


def combine_exact(G, e: np.ndarray, f: np.ndarray):
    """Exact C_ij = sum_g 2^(e_i + f_j + 4 - 8 g) G_g[i, j], returned as an
    object array of integers N and the exponent E0 with C = N 2^E0, where
    the common exponent is per entry: E0_ij = e_i + f_j + 4 - 8 gmax."""
    gmax = max(G)
    N = None
    for g, Gg in G.items():
        term = Gg.astype(object) * (1 << (8 * (gmax - g)))
        N = term if N is None else N + term
    E0 = (e[:, None] + f[None, :] + 4 - 8 * gmax).astype(np.int64)
    return N, E0


def to_fraction(N, E0, idx) -> Fraction:
    k = int(E0[idx])
    return Fraction(int(N[idx])) * (Fraction(2) ** k)


def ozaki_dd(A, B, S: int, mode: str = "all", out_limbs: int = 2):
    """The split-precision product rounded to `out_limbs` limbs (2: double-
    double, 4: quad-double), plus the exact pieces (N, E0) of the value
    before rounding.  A, B: FP64 arrays or limb tuples."""
    if isinstance(A, tuple):
        e, f = row_exponents(A[0]), col_exponents(B[0])
        DA, _ = split_rows_limbs(A, e, S)
        DB, _ = split_cols_limbs(B, f, S)
    else:
        e, f = row_exponents(A), col_exponents(B)
        DA, _ = split_rows(A, e, S)
        DB, _ = split_cols(B, f, S)
    G = group_sums(DA, DB, S, mode)
    N, E0 = combine_exact(G, e, f)
    C = tuple(np.zeros(N.shape) for _ in range(out_limbs))
    for idx in np.ndindex(N.shape):
        limbs = exact.round_to_limbs(to_fraction(N, E0, idx), out_limbs)
        for q in range(out_limbs):
            C[q][idx] = limbs[q]
    return C, (N, E0)


def apriori_unit(S: int, mode: str = "all") -> float:
    """Bound on |a b - (kept digit products)|, in units of 2^(e_i + f_j), for
    |a| < 2^e_i, |b| < 2^f_j cut into S digits: each remainder is below
    2^(e + 2 - 8S) and each kept part, a truncation, is below 2^e, so with
    all pairs the error is below 2^(3 - 8S); the triangle also drops, on
    each diagonal g = S+2 .. 2S, #pairs_g products of at most
    128^2 2^(4 - 8g) each."""
    b = 2.0 ** (3 - 8 * S)
    if mode == "triangle":
        for g in range(S + 2, 2 * S + 1):
            cnt = sum(1 for s in range(1, S + 1) if 1 <= g - s <= S)
            b += cnt * 128 * 128 * 2.0 ** (4 - 8 * g)
    return b


def apriori_bound(A: np.ndarray, B: np.ndarray, S: int, mode: str = "all"):
    """Per-entry bound on |C_S - AB|_ij from the truncated slices:
    l 2^(e_i + f_j) times apriori_unit(S, mode)."""
    l = A.shape[1]
    e, f = row_exponents(A), col_exponents(B)
    base = l * np.ldexp(1.0, (e[:, None] + f[None, :]).astype(np.int64))
    return base * apriori_unit(S, mode)


def slices_for_bits(bits: int, mode: str = "all", max_slices: int = 40) -> int:
    """Fewest slices whose a-priori bound is at most 2^-bits (per unit of
    l 2^(e_i + f_j)); 0 if even max_slices do not reach it."""
    for S in range(1, max_slices + 1):
        if apriori_unit(S, mode) <= 2.0 ** -bits:
            return S
    return 0
