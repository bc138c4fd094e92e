"""Split product through residues (the CRT form of the Ozaki scheme), plainly.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

Instead of products of digit planes, the integer images of the operands are
multiplied modulo several small pairwise coprime moduli and the exact integer
product is recovered by the Chinese remainder theorem:

1. row scale e_i of A and column scale f_j of B as in the digit form
   (smallest integer with every |a_ik| < 2^e_i, 0 for a zero line);
2. integer images with S radix-256 digits' worth of bits:
   A'_ik = trunc(a_ik 2^(8S - 2 - e_i)), |A'_ik| < 2^(8S - 2) (likewise B'),
   the value the S kept digits of the digit form add up to;
3. for each modulus p: residues of A' and B' in [-p/2, p/2) (they fit a
   signed byte for p <= 256), their integer product, and that product
   reduced to [0, p);
4. the CRT gives the unique X in [-P/2, P/2) (P the product of the moduli)
   with X = r_p mod p for every p; it equals (A' B')_ij whenever
   P > 2 max |(A' B')_ij|, which the moduli count is chosen for;
5. C_ij = X 2^(e_i + f_j + 4 - 16S), rounded to double-double.

The moduli are the pairwise coprime integers taken greedily from 256
downwards (the largest ones first, so few moduli carry many bits).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from oracle import exact, ozaki


def moduli(max_count: int = 64):
    out = []
    for x in range(256, 2, -1):
        if all(math.gcd(x, y) == 1 for y in out):
            out.append(x)
        if len(out) == max_count:
            break
    return out


def moduli_for_bits(bits: int):
    """Fewest leading moduli whose product exceeds 2^bits (None if the list
    is too short)."""
    P = 1
    for i, p in enumerate(moduli()):
        P *= p
        if P > (1 << bits):
            return i + 1
    return None


def product_bits(S: int, l: int) -> int:
    """Bits P must exceed: |(A' B')_ij| < l 2^(16S - 4), and the symmetric
    range needs P > 2 max |X|."""
    return 16 * S - 4 + max(l - 1, 0).bit_length() + 1


def images_rows(X, e: np.ndarray, S: int):
    """A'_ik = trunc(x_ik 2^(8S - 2 - e_i)) of the exact multi-limb values
    (object array of Python ints)."""
    R, K = X[0].shape
    out = np.zeros((R, K), dtype=object)
    for i in range(R):
        sc = Fraction(2) ** (8 * S - 2 - int(e[i]))
        for k in range(K):
            v = sum((Fraction(float(p[i, k])) for p in X), Fraction(0)) * sc
            out[i, k] = int(v)          # int() of a Fraction truncates toward zero
    return out


def images_cols(X, f: np.ndarray, S: int):
    return images_rows(tuple(np.ascontiguousarray(p.T) for p in X), f, S).T


def sym_mod(x, p: int):
    """x reduced into [-p/2, p/2) (elementwise on object arrays)."""
    return np.vectorize(lambda v: (int(v) + p // 2) % p - p // 2, otypes=[object])(x)


def crt(residues, mods):
    """The X in [-P/2, P/2) with X = r_j mod p_j for every j (residues: list
    of object arrays in [0, p_j))."""
    P = math.prod(mods)
    acc = np.zeros(residues[0].shape, dtype=object)
    for r, p in zip(residues, mods):
        M = P // p
        y = pow(M, -1, p)
        acc = acc + r * (M * y)
    acc = np.vectorize(lambda v: int(v) % P, otypes=[object])(acc)
    return np.vectorize(lambda v: v - P if 2 * v >= P else v, otypes=[object])(acc)


def crt_product(A, B, S: int, N: int | None = None, out_limbs: int = 2):
    """C = A B by the residue form with S digits' worth of bits per operand
    and N moduli (None: the fewest that hold the product).  A, B: tuples of
    limb planes.  Returns (C limb tuple, X, (e, f))."""
    e = ozaki.row_exponents(A[0])
    f = ozaki.col_exponents(B[0])
    l = A[0].shape[1]
    if N is None:
        N = moduli_for_bits(product_bits(S, l))
        if N is None:
            raise ValueError("product too wide for the moduli list")
    mods = moduli()[:N]
    Ai = images_rows(A, e, S)
    Bi = images_cols(B, f, S)
    res = []
    for p in mods:
        ra = np.array(sym_mod(Ai, p), dtype=np.int64)
        rb = np.array(sym_mod(Bi, p), dtype=np.int64)
        prod = ra @ rb                   # |entries| < l 2^14: exact in int64
        res.append(np.array(prod % p, dtype=object))
    X = crt(res, mods)
    m, n = X.shape
    C = [np.zeros((m, n)) for _ in range(out_limbs)]
    for i in range(m):
        for j in range(n):
            v = Fraction(int(X[i, j])) * Fraction(2) ** (int(e[i]) + int(f[j]) + 4 - 16 * S)
            for q, d in enumerate(exact.round_to_limbs(v, out_limbs)):
                C[q][i, j] = d
    return tuple(C), X, (e, f)
