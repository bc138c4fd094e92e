"""GPU parity of the double-double path (simple, block, Strassen) against the
oracle: exact AB from the oracle's super-accumulator or Python integers,
componentwise bound 8 l 2^-104 (|A||B|)_ij for simple and block, normwise
Winograd bound for Strassen."""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_1710_01839_amd import inputs
from tests.helpers import (error_ratio_exact_python, error_ratio_full, normwise_ratio,
                           sampled_errors, sampled_pairs, winograd_bound)

pytestmark = pytest.mark.gpu

DD_BOUND = 8.0            # |C - AB| <= 8 l 2^-104 (|A||B|)


def run_dd(M, ctx, A, B, algo="block", tile=None, out=None):
    Ad, Bd = M.to_device(A), M.to_device(B)
    m, n = A[0].shape[0], B[0].shape[1]
    C = out if out is not None else M.empty_like_limbs(m, n, 2)
    M.mpgemm_dd(ctx, Ad, Bd, C, algo=algo, tile=tile)
    torch.cuda.synchronize()
    return M.to_host(C)


def test_config0_simple_128_exact_python(gpu):
    """m = l = n = 128, simple triple loop, all entries vs Python integers."""
    M, ctx = gpu
    A, B = inputs.dd_uniform(128, 128, 0), inputs.dd_uniform(128, 128, 1)
    C = run_dd(M, ctx, A, B, "simple")
    r = error_ratio_exact_python(C, A, B, -104)
    print("config0 simple ratio", r)
    assert r <= DD_BOUND


@pytest.mark.parametrize("dist", ["uniform", "illcond"])
def test_block_variants_ragged(gpu, dist):
    """Every built tile variant on a ragged shape spanning several tiles."""
    M, ctx = gpu
    gen = inputs.dd_uniform if dist == "uniform" else inputs.dd_illcond
    m, n, l = 203, 141, 157
    A, B = gen(m, l, 2), gen(l, n, 3)
    ref = run_dd(M, ctx, A, B, "simple")
    r, _ = error_ratio_full(ref, A, B, -104)
    print(dist, "simple ratio", r)
    assert r <= DD_BOUND
    for v in M.variants(2):
        C = run_dd(M, ctx, A, B, "block", v)
        # same operation sequence per entry as the simple kernel
        assert np.array_equal(C[0], ref[0]) and np.array_equal(C[1], ref[1]), v


def _direct_variants(M):
    """The variant whose operand tiles the load unit moves to LDS (64x64x8,
    2x4 per thread, 512 threads)."""
    vs = [v for v in M.variants(2) if (v["bm"], v["bn"], v["bk"], v["tm"], v["tn"]) == (64, 64, 8, 2, 4)]
    assert len(vs) == 1
    return vs


def _padded_view(X, extra, fill):
    """Device copies of the limbs inside wider buffers (extra columns = fill)."""
    out = []
    for x in X:
        buf = torch.full((x.shape[0], x.shape[1] + extra), fill, dtype=torch.float64, device="cuda")
        buf[:, :x.shape[1]] = torch.from_numpy(x).cuda()
        out.append(buf[:, :x.shape[1]])
    return tuple(out)


@pytest.mark.parametrize("shape", [(203, 142, 158), (64, 64, 8), (1, 2, 2), (130, 66, 520), (65, 64, 10)])
def test_direct_variants_ragged(gpu, shape):
    """Load-unit-to-LDS variants on shapes meeting their alignment (n, l
    even) with tails in every dimension, also on operands that are views
    into wider buffers whose extra columns hold NaN: out-of-range chunks must
    be zero-filled, never read.  Bit-identical to the simple kernel."""
    M, ctx = gpu
    m, n, l = shape
    A, B = inputs.dd_uniform(m, l, 12), inputs.dd_uniform(l, n, 13)
    ref = run_dd(M, ctx, A, B, "simple")
    for v in _direct_variants(M):
        C = run_dd(M, ctx, A, B, "block", v)
        assert np.array_equal(C[0], ref[0]) and np.array_equal(C[1], ref[1]), v
        Ad, Bd = _padded_view(A, 6, float("nan")), _padded_view(B, 4, float("nan"))
        Cd = M.empty_like_limbs(m, n, 2)
        M.mpgemm_dd(ctx, Ad, Bd, Cd, algo="block", tile=v)
        torch.cuda.synchronize()
        C = M.to_host(Cd)
        assert np.array_equal(C[0], ref[0]) and np.array_equal(C[1], ref[1]), (v, "padded")


def test_direct_variants_fallback(gpu):
    """Odd l or n (or odd leading dimensions) take the register-staged
    kernel of the same tile: results stay bit-identical."""
    M, ctx = gpu
    for (m, n, l) in ((70, 63, 40), (70, 64, 41)):
        A, B = inputs.dd_uniform(m, l, 14), inputs.dd_uniform(l, n, 15)
        ref = run_dd(M, ctx, A, B, "simple")
        for v in _direct_variants(M):
            C = run_dd(M, ctx, A, B, "block", v)
            assert np.array_equal(C[0], ref[0]) and np.array_equal(C[1], ref[1]), (v, m, n, l)


def test_integer_inputs_bit_exact(gpu):
    """Integer inputs |x| <= 2^30: every step is exact, so the result is the
    canonical DD of the integer product, bit for bit."""
    M, ctx = gpu
    m, n, l = 70, 90, 300
    A = inputs.integers(m, l, 2, 4)
    B = inputs.integers(l, n, 2, 5)
    Ce = cref.gemm_exact(A, B, out_limbs=2)
    for algo, tile in (("simple", None), ("block", None), ("block", M.variants(2)[4]),
                       ("strassen", {"depth": 1}), ("strassen", {"depth": 2})):
        C = run_dd(M, ctx, A, B, algo, tile)
        assert np.array_equal(C[0], Ce[0]) and np.array_equal(C[1], Ce[1]), (algo, tile)


def test_paper_matrices_closed_form(gpu):
    """A = [sqrt5 (i+j-1)], B = [sqrt3 (n-i)] (the paper's test matrices):
    c_ij = sqrt15 n(n-1)(3i+n-2)/6, independent of j."""
    M, ctx = gpu
    n = 96
    A, B = inputs.paper_matrices(n, 2)
    C = run_dd(M, ctx, A, B, "block")
    r, _ = error_ratio_full(C, A, B, -104)
    assert r <= DD_BOUND
    # closed form, evaluated exactly with integer square roots
    from fractions import Fraction
    import math
    for i in (1, 17, n):
        v = Fraction(n * (n - 1) * (3 * i + n - 2), 6)
        # sqrt(15) * v to ~200 bits
        ref = Fraction(math.isqrt(15 * (v.numerator ** 2) * 4 ** 200), v.denominator * 2 ** 200)
        got = Fraction(C[0][i - 1, 5]) + Fraction(C[1][i - 1, 5])
        # input rounding (2 ulp of DD) plus the GEMM bound
        assert abs(got - ref) <= ref * Fraction(1, 2 ** 90)
        assert C[0][i - 1, 0] == C[0][i - 1, n - 1] and C[1][i - 1, 0] == C[1][i - 1, n - 1]


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_normwise(gpu, depth):
    M, ctx = gpu
    n = 256
    A, B = inputs.dd_uniform(n, n, 6), inputs.dd_uniform(n, n, 7)
    C = run_dd(M, ctx, A, B, "strassen", {"depth": depth})
    r = normwise_ratio(C, A, B, 2)
    bound = winograd_bound(n, depth, 8 * 2.0 ** -104)
    print("strassen depth", depth, "normwise", r, "bound", bound)
    assert r <= bound


def test_strassen_ragged(gpu):
    """Odd, non-square dimensions are zero-padded to a multiple of 2^depth."""
    M, ctx = gpu
    m, n, l = 131, 77, 101
    A, B = inputs.dd_uniform(m, l, 8), inputs.dd_uniform(l, n, 9)
    for d in (1, 2):
        C = run_dd(M, ctx, A, B, "strassen", {"depth": d})
        r = normwise_ratio(C, A, B, 2)
        assert r <= winograd_bound(max(m, n, l) + 4, d, 8 * 2.0 ** -104)


def test_strided_leading_dimensions(gpu):
    """lda > l, ldb > n, ldc > n (views into larger buffers)."""
    M, ctx = gpu
    m, n, l = 65, 70, 33
    A, B = inputs.dd_uniform(m, l + 7, 10), inputs.dd_uniform(l, n + 5, 11)
    Ad = M.to_device(A)
    Bd = M.to_device(B)
    Av = tuple(x[:, :l] for x in Ad)
    Bv = tuple(x[:, :n] for x in Bd)
    Cbig = tuple(torch.full((m, n + 9), 7.0, dtype=torch.float64, device="cuda") for _ in range(2))
    Cv = tuple(x[:, :n] for x in Cbig)
    M.mpgemm_dd(ctx, Av, Bv, Cv, algo="block")
    torch.cuda.synchronize()
    C = M.to_host(Cv)
    Ah = tuple(np.ascontiguousarray(x[:, :l]) for x in A)
    Bh = tuple(np.ascontiguousarray(x[:, :n]) for x in B)
    r, _ = error_ratio_full(tuple(np.ascontiguousarray(c) for c in C), Ah, Bh, -104)
    assert r <= DD_BOUND
    pad = Cbig[0][:, n:].cpu().numpy()
    assert np.all(pad == 7.0)  # nothing written outside the m x n view


def test_edge_cases(gpu):
    M, ctx = gpu
    # 1 x 1 x 1
    A, B = inputs.dd_uniform(1, 1, 12), inputs.dd_uniform(1, 1, 13)
    C = run_dd(M, ctx, A, B, "block")
    Ce = cref.gemm_exact(A, B, out_limbs=2)
    assert abs((C[0][0, 0] - Ce[0][0, 0]) + (C[1][0, 0] - Ce[1][0, 0])) <= 2.0 ** -100 * abs(Ce[0][0, 0])
    # l == 0 sets C = 0
    Ad = tuple(torch.empty((5, 0), dtype=torch.float64, device="cuda") for _ in range(2))
    Bd = tuple(torch.empty((0, 6), dtype=torch.float64, device="cuda") for _ in range(2))
    Cd = tuple(torch.full((5, 6), 3.0, dtype=torch.float64, device="cuda") for _ in range(2))
    M.mpgemm_dd(ctx, Ad, Bd, Cd)
    torch.cuda.synchronize()
    assert float(Cd[0].abs().max()) == 0.0 and float(Cd[1].abs().max()) == 0.0
    # m == 0 is a no-op
    Ad = tuple(torch.empty((0, 4), dtype=torch.float64, device="cuda") for _ in range(2))
    Bd = tuple(torch.ones((4, 3), dtype=torch.float64, device="cuda") for _ in range(2))
    Cd = tuple(torch.empty((0, 3), dtype=torch.float64, device="cuda") for _ in range(2))
    M.mpgemm_dd(ctx, Ad, Bd, Cd)


def test_errors_are_reported(gpu):
    M, ctx = gpu
    A = M.to_device(inputs.dd_uniform(8, 8, 14))
    B = M.to_device(inputs.dd_uniform(8, 8, 15))
    C = M.empty_like_limbs(8, 8, 2)
    with pytest.raises(M.MpgemmError) as e:
        M.mpgemm_dd(ctx, A, B, (A[0], C[1]))           # C aliases A
    assert e.value.status == M.MPG_ERR_ALIAS
    with pytest.raises(M.MpgemmError) as e:
        M.mpgemm_dd(ctx, A, B, C, algo="block", tile={"bm": 48, "bn": 48})
    assert e.value.status == M.MPG_ERR_UNSUPPORTED
    with pytest.raises(M.MpgemmError) as e:
        M.mpgemm_dd(ctx, A, B, C, algo="strassen", tile={"depth": 9})
    assert e.value.status == M.MPG_ERR_ARG


def test_deterministic(gpu):
    M, ctx = gpu
    A, B = inputs.dd_illcond(300, 200, 16), inputs.dd_illcond(200, 260, 17)
    for algo, tile in (("block", None), ("strassen", {"depth": 2})):
        C1 = run_dd(M, ctx, A, B, algo, tile)
        C2 = run_dd(M, ctx, A, B, algo, tile)
        assert np.array_equal(C1[0], C2[0]) and np.array_equal(C1[1], C2[1])


@pytest.mark.parametrize("algo,tile", [("block", None), ("block", "staged"), ("strassen", {"depth": 1}),
                                       ("strassen", {"depth": 2})])
def test_full_size_4096_sampled(gpu, algo, tile):
    """n = 4096, the benchmark's launch configuration (Strassen depth 2 over
    the default, direct tile): exact error at sampled entries (corners,
    random) against Python integers."""
    M, ctx = gpu
    n = 4096
    if tile == "staged":
        tile = M.variants(2)[0]      # the register-staged 64x64x16 kernel
    A, B = inputs.dd_uniform(n, n, 20), inputs.dd_uniform(n, n, 21)
    C = run_dd(M, ctx, A, B, algo, tile)
    pairs = sampled_pairs(n, n, 48)
    errs, mags = sampled_errors(C, A, B, pairs)
    if algo == "block":
        r = max(e / (n * 2.0 ** -104 * g) for e, g in zip(errs, mags))
        print(algo, "sampled componentwise ratio", r)
        assert r <= DD_BOUND
    else:
        amax = float(np.abs(A[0]).max()) * (1 + 2.0 ** -50)
        bmax = float(np.abs(B[0]).max()) * (1 + 2.0 ** -50)
        r = max(errs) / (amax * bmax)
        bound = winograd_bound(n, tile["depth"], 8 * 2.0 ** -104)
        print(algo, tile, "sampled normwise", r, "bound", bound)
        assert r <= bound
