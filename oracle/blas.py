"""Exact BLAS-style product C := alpha op(A) op(B) + beta C, written out plainly.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

The product op(A) op(B) is Eq. (1) of the paper; the surrounding form is the
standard xGEMM definition of the BLAS:

* op(X) is X ('N'), its transpose ('T') or its conjugate transpose ('C'; the
  transpose for real matrices);
* alpha and beta are multi-limb scalars; when beta == 0 the old C takes no
  part (its value, even NaN, is not read) and when alpha == 0 or the inner
  dimension is 0 the product takes no part.

Real matrices are tuples of limb planes; a complex matrix is a pair
(real part planes, imaginary part planes).  Everything is computed exactly in
Python integers on one common power-of-two scale; the result is returned
unrounded, as integers and their scale, together with the exact magnitudes
that the rounding-error bounds of a floating-point evaluation are stated in.
"""
from __future__ import annotations

import numpy as np

from oracle import exact

_iabs = np.vectorize(abs, otypes=[object])


def op(planes, trans: str):
    """op(X) of a limb-plane tuple: a view, nothing is copied or rounded."""
    if trans == "N":
        return tuple(planes)
    if trans in ("T", "C"):
        return tuple(np.ascontiguousarray(p.T) for p in planes)
    raise ValueError(trans)


def _scalar_int(limbs):
    """A multi-limb scalar as (integer, scale): value == M * 2^-s."""
    planes = [np.array([[float(x)]]) for x in limbs]
    s = exact.scale_of(planes)
    return int(exact.to_int(planes, s)[0, 0]), s


def _ints(planes):
    s = exact.scale_of(planes)
    return exact.to_int(planes, s), s


def _align(terms):
    """terms: list of (object array or int, scale).  Returns them on the
    largest scale, as a list of object arrays (or ints), and that scale."""
    S = max(s for _, s in terms)
    return [v * (1 << (S - s)) for v, s in terms], S


def rgemm_exact(transa: str, transb: str, alpha, A, B, beta, C):
    """Real form.  A, B, C: limb-plane tuples (A is stored so that op(A) is
    m x k, B so that op(B) is k x n, C is m x n).  alpha, beta: sequences of
    limbs.  Returns (R, mag_ab, mag_c, s): exact integer arrays with
    R 2^-s = alpha op(A) op(B) + beta C,
    mag_ab 2^-s = |alpha| |op(A)| |op(B)|, mag_c 2^-s = |beta| |C|."""
    a_int, sa = _scalar_int(alpha)
    b_int, sb = _scalar_int(beta)
    m, n = C[0].shape
    zero = np.zeros((m, n), dtype=object)
    opA, opB = op(A, transa), op(B, transb)
    k = opA[0].shape[1]
    assert opA[0].shape[0] == m and opB[0].shape == (k, n)
    if a_int == 0 or k == 0:
        P, Pabs, sp = zero, zero, 0
    else:
        Ai, sA = _ints(opA)
        Bi, sB = _ints(opB)
        P, Pabs, sp = Ai.dot(Bi), _iabs(Ai).dot(_iabs(Bi)), sA + sB
    if b_int == 0:
        Ci, sc = zero, 0
    else:
        Ci, sc = _ints(C)
    (t1, t2, t3, t4), s = _align([(a_int * P, sa + sp), (b_int * Ci, sb + sc),
                                  (abs(a_int) * Pabs, sa + sp), (_iabs(b_int * Ci), sb + sc)])
    return t1 + t2, t3, t4, s


def _cop(Z, trans: str):
    """op of a complex matrix (re planes, im planes): conjugation negates
    every limb of the imaginary part (exact)."""
    re, im = op(Z[0], trans), op(Z[1], trans)
    if trans == "C":
        im = tuple(-p for p in im)
    return re, im


def zgemm_exact(transa: str, transb: str, alpha, A, B, beta, C):
    """Complex form.  A, B, C: (re planes, im planes); alpha, beta:
    (re limbs, im limbs).  Returns (R_re, R_im, mag_ab, mag_c, s) with
    (R_re + i R_im) 2^-s = alpha op(A) op(B) + beta C exactly, and
    mag_ab 2^-s = (|ar| + |ai|) (|Ar| + |Ai|)(|Br| + |Bi|),
    mag_c 2^-s = (|br| + |bi|) (|Cr| + |Ci|), elementwise bounds of the
    moduli of the two parts that hold for both components."""
    ar, sar = _scalar_int(alpha[0])
    ai, sai = _scalar_int(alpha[1])
    br, sbr = _scalar_int(beta[0])
    bi, sbi = _scalar_int(beta[1])
    (ar, ai), sal = _align([(ar, sar), (ai, sai)])
    (br, bi), sbe = _align([(br, sbr), (bi, sbi)])
    m, n = C[0][0].shape
    zero = np.zeros((m, n), dtype=object)
    Ar, Ai = _cop(A, transa)
    Br, Bi = _cop(B, transb)
    k = Ar[0].shape[1]
    if (ar == 0 and ai == 0) or k == 0:
        Pr, Pi, Pm, sp = zero, zero, zero, 0
    else:
        (Ari, Aii), sA = _align([_ints(Ar), _ints(Ai)])
        (Bri, Bii), sB = _align([_ints(Br), _ints(Bi)])
        Pr = Ari.dot(Bri) - Aii.dot(Bii)
        Pi = Ari.dot(Bii) + Aii.dot(Bri)
        Pm = (_iabs(Ari) + _iabs(Aii)).dot(_iabs(Bri) + _iabs(Bii))
        sp = sA + sB
    if br == 0 and bi == 0:
        Cr, Ci, sc = zero, zero, 0
    else:
        (Cr, Ci), sc = _align([_ints(C[0]), _ints(C[1])])
    re_ab, im_ab = ar * Pr - ai * Pi, ar * Pi + ai * Pr
    re_c, im_c = br * Cr - bi * Ci, br * Ci + bi * Cr
    mag_ab = (abs(ar) + abs(ai)) * Pm
    mag_c = (abs(br) + abs(bi)) * (_iabs(Cr) + _iabs(Ci))
    (x1, x2, x3, x4, x5, x6), s = _align([(re_ab, sal + sp), (im_ab, sal + sp), (re_c, sbe + sc),
                                          (im_c, sbe + sc), (mag_ab, sal + sp), (mag_c, sbe + sc)])
    return x1 + x3, x2 + x4, x5, x6, s


def error_over_bound(Cout, R, mag_ab, mag_c, s, coef_ab, coef_c, unit_exp: int):
    """max over elements of |Cout - R 2^-s| / ((coef_ab mag_ab + coef_c mag_c)
    2^(unit_exp - s)), computed exactly (inf where the bound is 0 and the
    element is not exact).  Cout: limb-plane tuple of the computed result."""
    from fractions import Fraction
    sC = max(s, exact.scale_of(Cout))
    G = exact.to_int(Cout, sC)
    up = 1 << (sC - s)
    worst = 0.0
    for idx in np.ndindex(Cout[0].shape):
        err = abs(int(G[idx]) - int(R[idx]) * up)
        bound = Fraction(coef_ab * int(mag_ab[idx]) + coef_c * int(mag_c[idx])) * up * Fraction(2) ** unit_exp
        if bound == 0:
            r = 0.0 if err == 0 else float("inf")
        else:
            r = float(Fraction(err) / bound)
        worst = max(worst, r)
    return worst
