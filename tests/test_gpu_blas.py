"""GPU parity of the BLAS-style form C := alpha op(A) op(B) + beta C (real DD,
real QD, complex DD) against the exact oracle of that form, with the
componentwise bounds stated for mpg_rgemm / mpg_zgemm_dd, plus bitwise
agreement with the plain product on explicitly transposed copies, the
special cases of the form and the argument checks."""
import ctypes
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import blas
from paper_1710_01839_amd import inputs

pytestmark = pytest.mark.gpu


def stored(rows, cols, trans, seed, limbs=2, pad=0):
    """Limb planes holding an operand whose op() is rows x cols, stored with
    `pad` extra columns (leading dimension > width)."""
    r, c = (rows, cols) if trans == "N" else (cols, rows)
    X = inputs.dd_illcond(r, c + pad, seed_offset=seed, kmax=6) if limbs == 2 else \
        inputs.qd_uniform(r, c + pad, seed_offset=seed)
    return X, tuple(np.ascontiguousarray(p[:, :c]) for p in X)


def dev_padded(X, width):
    """Device planes with a leading dimension of X's full width, viewed at
    `width` columns."""
    return tuple(torch.as_tensor(p, device="cuda")[:, :width] for p in X)


def real_ratio(C, ta, tb, alpha, A, B, beta, Cin, k, unit_exp):
    R, mab, mc, s = blas.rgemm_exact(ta, tb, alpha, A, B, beta, Cin)
    return blas.error_over_bound(C, R, mab, mc, s, 8 * k + 16, 16, unit_exp)


SCALARS = [((1.0, 0.0), (0.0, 0.0)),
           ((-2.5, 2.0 ** -60), (0.75, -2.0 ** -57)),
           ((1.0 / 3, 1.0 / 3 * 2.0 ** -54), (0.0, 0.0))]


@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("sc", range(len(SCALARS)))
def test_real_dd_form(gpu, ta, tb, sc):
    """Ragged m, n, k over several 64-wide tiles, padded leading dimensions;
    beta == 0 cases run with NaN in C (it must not be read)."""
    M, ctx = gpu
    m, n, k = 67, 45, 83
    alpha, beta = SCALARS[sc]
    Af, A = stored(m, k, ta, 1, pad=3)
    Bf, B = stored(k, n, tb, 2, pad=5)
    Cin = inputs.dd_illcond(m, n, seed_offset=3, kmax=6)
    Cd = M.to_device(Cin)
    if beta == (0.0, 0.0):
        Cd[0].fill_(float("nan"))
    M.rgemm(ctx, dev_padded(Af, A[0].shape[1]), dev_padded(Bf, B[0].shape[1]), Cd, alpha, beta,
            ta, tb)
    torch.cuda.synchronize()
    r = real_ratio(M.to_host(Cd), ta, tb, alpha, A, B, beta, Cin, k, -104)
    print(ta, tb, sc, "ratio", r)
    assert r <= 1.0


@pytest.mark.parametrize("ta,tb,algo", [("T", "N", "block"), ("N", "T", "block"), ("T", "T", "block"),
                                        ("T", "T", "ozaki_crt")])
def test_real_qd_form(gpu, ta, tb, algo):
    """QD form; the residue-form product (three exact part products) meets
    the same bound."""
    M, ctx = gpu
    m, n, k = 37, 29, 41
    alpha = (-0.75, 2.0 ** -58, -2.0 ** -112, 2.0 ** -166)
    beta = (1.5, -2.0 ** -54, 2.0 ** -108, 0.0)
    _, A = stored(m, k, ta, 4, limbs=4)
    _, B = stored(k, n, tb, 5, limbs=4)
    Cin = inputs.qd_uniform(m, n, seed_offset=6)
    Cd = M.to_device(Cin)
    M.rgemm(ctx, M.to_device(A), M.to_device(B), Cd, alpha, beta, ta, tb, algo)
    torch.cuda.synchronize()
    r = real_ratio(M.to_host(Cd), ta, tb, alpha, A, B, beta, Cin, k, -208)
    print(ta, tb, "qd ratio", r)
    assert r <= 1.0


@pytest.mark.parametrize("algo,tile", [("block", None), ("simple", None),
                                       ("strassen", {"depth": 1}), ("ozaki", {"slices": 0}),
                                       ("ozaki_crt", {"slices": 0})])
def test_transposes_are_bitwise_the_plain_product(gpu, algo, tile):
    """op(A) op(B) with alpha = 1, beta = 0 is the plain product of the
    transposed copies, bit for bit, for every algorithm; with alpha and beta
    the result equals the same call on untransposed copies."""
    M, ctx = gpu
    m, n, k = 130, 98, 150
    _, At = stored(m, k, "T", 7)
    _, Bt = stored(k, n, "T", 8)
    A = tuple(np.ascontiguousarray(p.T) for p in At)
    B = tuple(np.ascontiguousarray(p.T) for p in Bt)
    C1 = M.empty_like_limbs(m, n, 2)
    C2 = M.empty_like_limbs(m, n, 2)
    M.rgemm(ctx, M.to_device(At), M.to_device(Bt), C1, 1.0, 0.0, "T", "T", algo, tile)
    M.mpgemm_dd(ctx, M.to_device(A), M.to_device(B), C2, algo, tile)
    torch.cuda.synchronize()
    for p, q in zip(M.to_host(C1), M.to_host(C2)):
        assert np.array_equal(p, q)
    Cin = inputs.dd_uniform(m, n, seed_offset=9)
    C3, C4 = M.to_device(Cin), M.to_device(Cin)
    M.rgemm(ctx, M.to_device(At), M.to_device(B), C3, (0.5, 2.0 ** -70), (-3.0, 0.0), "T", "N",
            algo, tile)
    M.rgemm(ctx, M.to_device(A), M.to_device(B), C4, (0.5, 2.0 ** -70), (-3.0, 0.0), "N", "N",
            algo, tile)
    torch.cuda.synchronize()
    for p, q in zip(M.to_host(C3), M.to_host(C4)):
        assert np.array_equal(p, q)


ZALPHA = ((0.75, 2.0 ** -56), (-1.5, 0.0))
ZBETA = ((-0.5, 0.0), (2.0, -2.0 ** -55))


def zflat(s):
    return (s[0][0], s[0][1], s[1][0], s[1][1])


def cplx(rows, cols, trans, seed):
    _, re = stored(rows, cols, trans, seed)
    _, im = stored(rows, cols, trans, seed + 1)
    return re, im


@pytest.mark.parametrize("ta,tb", list(itertools.product("NTC", "NTC")))
def test_complex_dd_form(gpu, ta, tb):
    M, ctx = gpu
    m, n, k = 35, 27, 39
    A = cplx(m, k, ta, 11)
    B = cplx(k, n, tb, 13)
    Cin = (inputs.dd_uniform(m, n, seed_offset=15), inputs.dd_uniform(m, n, seed_offset=16))
    Cd = M.to_device(Cin[0] + Cin[1])
    M.zgemm_dd(ctx, M.to_device(A[0] + A[1]), M.to_device(B[0] + B[1]), Cd, zflat(ZALPHA),
               zflat(ZBETA), ta, tb)
    torch.cuda.synchronize()
    out = M.to_host(Cd)
    Rr, Ri, mab, mc, s = blas.zgemm_exact(ta, tb, ZALPHA, A, B, ZBETA, Cin)
    rr = blas.error_over_bound(out[:2], Rr, mab, mc, s, 16 * k + 32, 32, -104)
    ri = blas.error_over_bound(out[2:], Ri, mab, mc, s, 16 * k + 32, 32, -104)
    print(ta, tb, "complex ratios", rr, ri)
    assert rr <= 1.0 and ri <= 1.0


@pytest.mark.parametrize("algo,tile", [("strassen", {"depth": 1}), ("ozaki", {"slices": 0}),
                                       ("ozaki_crt", {"slices": 0})])
def test_complex_other_products(gpu, algo, tile):
    """The embedding's product by Strassen or by the split product: a
    double-double-level normwise check, 2^-96 max|.| (|A||B|) per term."""
    M, ctx = gpu
    m, n, k = 96, 80, 112
    A = cplx(m, k, "C", 21)
    B = cplx(k, n, "T", 23)
    Cd = M.empty_like_limbs(m, n, 4)
    one, zero = ((1.0, 0.0), (0.0, 0.0)), ((0.0, 0.0), (0.0, 0.0))
    M.zgemm_dd(ctx, M.to_device(A[0] + A[1]), M.to_device(B[0] + B[1]), Cd, zflat(one),
               zflat(zero), "C", "T", algo, tile)
    torch.cuda.synchronize()
    out = M.to_host(Cd)
    Rr, Ri, mab, mc, s = blas.zgemm_exact("C", "T", one, A, B, zero, (out[:2], out[2:]))
    big = max(int(v) for v in mab.flat)
    norm = np.full(mab.shape, big, dtype=object)
    rr = blas.error_over_bound(out[:2], Rr, norm, mc, s, 2 * k, 0, -96)
    ri = blas.error_over_bound(out[2:], Ri, norm, mc, s, 2 * k, 0, -96)
    print(algo, "complex normwise ratios", rr, ri)
    assert rr <= 1.0 and ri <= 1.0


def test_special_cases(gpu):
    """alpha == 0 (A and B hold NaN and are not read), k == 0, m == 0."""
    M, ctx = gpu
    m, n, k = 20, 30, 10
    Cin = inputs.dd_uniform(m, n, seed_offset=31)
    nanA = (torch.full((m, k), float("nan"), dtype=torch.float64, device="cuda"),
            torch.zeros((m, k), dtype=torch.float64, device="cuda"))
    nanB = (torch.full((k, n), float("nan"), dtype=torch.float64, device="cuda"),
            torch.zeros((k, n), dtype=torch.float64, device="cuda"))
    Cd = M.to_device(Cin)
    M.rgemm(ctx, nanA, nanB, Cd, 0.0, (0.5, 0.0))
    torch.cuda.synchronize()
    h = M.to_host(Cd)
    assert np.array_equal(h[0], Cin[0] / 2) and np.array_equal(h[1], Cin[1] / 2)
    empty = M.empty_like_limbs(m, 0, 2), M.empty_like_limbs(0, n, 2)
    Cd = M.to_device(Cin)
    M.rgemm(ctx, empty[0], empty[1], Cd, 3.0, (-2.0, 0.0))
    torch.cuda.synchronize()
    h = M.to_host(Cd)
    assert np.array_equal(h[0], -2 * Cin[0]) and np.array_equal(h[1], -2 * Cin[1])
    Cd = M.to_device(Cin)
    M.rgemm(ctx, empty[0], empty[1], Cd, 3.0, 0.0)
    torch.cuda.synchronize()
    assert all(not p.any() for p in M.to_host(Cd))
    # complex: alpha == 0 with NaN inputs; beta == 0 with NaN in C
    Z = M.to_device(Cin + Cin)
    zA = nanA + nanA
    zB = nanB + nanB
    M.zgemm_dd(ctx, zA, zB, Z, (0.0,) * 4, (0.0, 0.0, 1.0, 0.0))   # C := i C
    torch.cuda.synchronize()
    h = M.to_host(Z)
    assert np.array_equal(h[0], -Cin[0]) and np.array_equal(h[2], Cin[0])
    A = cplx(m, k, "N", 33)
    B = cplx(k, n, "N", 35)
    Z = M.empty_like_limbs(m, n, 4)
    for p in Z:
        p.fill_(float("nan"))
    M.zgemm_dd(ctx, M.to_device(A[0] + A[1]), M.to_device(B[0] + B[1]), Z)
    torch.cuda.synchronize()
    assert all(np.isfinite(p).all() for p in M.to_host(Z))
    # m == 0 is a no-op
    M.rgemm(ctx, M.empty_like_limbs(0, k, 2), M.empty_like_limbs(k, n, 2),
            M.empty_like_limbs(0, n, 2), 1.0, 0.0)


def test_argument_errors(gpu):
    M, ctx = gpu
    L = M._lib
    A = M.empty_like_limbs(8, 8, 2)
    B = M.empty_like_limbs(8, 8, 2)
    C = M.empty_like_limbs(8, 8, 2)
    pa, _ = M._limb_array(A)
    pb, _ = M._limb_array(B)
    pc, _ = M._limb_array(C)
    one = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 0.0)
    zero = (ctypes.c_double * 4)()
    po, pz = ctypes.cast(one, M._pd), ctypes.cast(zero, M._pd)

    def call(prec=2, ta=0, tb=0, m=8, n=8, k=8, lda=8, ldb=8, ldc=8, pa=pa, pc=pc, algo=2):
        return L.mpg_rgemm(ctx.handle, prec, ta, tb, m, n, k, po, pa, lda, pb, ldb, pz, pc, ldc,
                           algo, None)

    assert call() == M.MPG_OK
    assert call(prec=3) == M.MPG_ERR_ARG
    assert call(ta=5) == M.MPG_ERR_ARG
    assert call(lda=7) == M.MPG_ERR_ARG
    assert call(ta=1, m=4, lda=3) == M.MPG_ERR_ARG          # stored k x m needs lda >= m
    assert call(ldc=7) == M.MPG_ERR_ARG
    assert call(k=-1) == M.MPG_ERR_ARG
    assert call(pc=pa) == M.MPG_ERR_ALIAS
    big = M.empty_like_limbs(8, 8, 4)
    p4, _ = M._limb_array(big)
    assert L.mpg_rgemm(ctx.handle, 4, 0, 0, 8, 8, 8, po, p4, 8, p4, 8, pz, p4, 8, 2, None) == \
        M.MPG_ERR_ALIAS
    keep = [M.empty_like_limbs(8, 8, 4) for _ in range(3)]   # distinct live buffers
    q4a, q4b, q4c = (M._limb_array(x)[0] for x in keep)
    assert L.mpg_rgemm(ctx.handle, 4, 0, 0, 8, 8, 8, po, q4a, 8, q4b, 8, pz, q4c, 8, 4, None) == \
        M.MPG_ERR_UNSUPPORTED
    assert L.mpg_zgemm_dd(ctx.handle, 0, 0, 8, 8, (1 << 30) + 1, po, q4a, 8, q4b, 8, pz, q4c, 8,
                          2, None) == M.MPG_ERR_ARG
    torch.cuda.synchronize()


def test_full_size_transposed(gpu):
    """m = n = k = 4096, both operands transposed, alpha and beta: bitwise the
    untransposed call on transposed copies, and sampled entries against the
    exact form."""
    M, ctx = gpu
    nn = 4096
    At = inputs.dd_uniform(nn, nn, 41)
    Bt = inputs.dd_uniform(nn, nn, 42)
    Cin = inputs.dd_uniform(nn, nn, 43)
    alpha, beta = (-1.25, 2.0 ** -62), (0.5, 0.0)
    C1 = M.to_device(Cin)
    M.rgemm(ctx, M.to_device(At), M.to_device(Bt), C1, alpha, beta, "T", "T", "strassen",
            {"depth": 2})
    Ad = tuple(t.t().contiguous() for t in M.to_device(At))
    Bd = tuple(t.t().contiguous() for t in M.to_device(Bt))
    C2 = M.to_device(Cin)
    M.rgemm(ctx, Ad, Bd, C2, alpha, beta, "N", "N", "strassen", {"depth": 2})
    torch.cuda.synchronize()
    for p, q in zip(C1, C2):
        assert torch.equal(p, q)
    out = M.to_host(C1)
    g = np.random.default_rng(44)
    rows = sorted({0, nn - 1, *map(int, g.integers(0, nn, 6))})
    cols = sorted({0, nn - 1, *map(int, g.integers(0, nn, 6))})
    A = tuple(np.ascontiguousarray(p[:, rows].T) for p in At)      # rows of op(A)
    B = tuple(np.ascontiguousarray(p[cols, :].T) for p in Bt)      # columns of op(B)
    Cs = tuple(np.ascontiguousarray(p[np.ix_(rows, cols)]) for p in Cin)
    R, mab, mc, s = blas.rgemm_exact("N", "N", alpha, A, B, beta, Cs)
    got = tuple(np.ascontiguousarray(p[np.ix_(rows, cols)]) for p in out)
    # Strassen depth 2 over the block kernel: the normwise Winograd bound in
    # units of 2^-104 max|A| max|B| (scaled by |alpha|), plus the epilogue
    n0 = nn / 4
    wino = 18 ** 2 * (n0 * n0 + 6 * n0) - 6 * nn
    amax = max(float(np.abs(At[0]).max()), float(np.abs(Bt[0]).max())) * (1 + 2.0 ** -50)
    V = Fraction(wino) * Fraction(1.25 + 2.0 ** -50) * Fraction(amax) ** 2
    norm = np.full(mab.shape, math.ceil(V * (1 << s)), dtype=object)
    r = blas.error_over_bound(got, R, norm, mc, s, 1, 16, -104)
    print("n=4096 TT strassen2 sampled ratio", r)
    assert r <= 1.0
