"""Split-K (MPG_SPLITK) against the oracle: the K range cut into chunks whose
partial products are added in a fixed order (Eq. (1) and Eq. (2) fix no
order of summation).  Componentwise DD / QD bounds against the exact
product, run-to-run bitwise determinism, bit-exact integer results, ragged
last chunks, dot-product shapes, the tuning table and the tuner."""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_1710_01839_amd import inputs
from tests.helpers import ExactSample, error_ratio_full

pytestmark = pytest.mark.gpu

DD_BOUND = 8.0            # |C - AB| <= 8 l 2^-104 (|A||B|)


def run(M, ctx, A, B, tile=None, algo="splitk"):
    L = len(A)
    m, n = A[0].shape[0], B[0].shape[1]
    C = M.empty_like_limbs(m, n, L)
    f = M.mpgemm_dd if L == 2 else M.mpgemm_qd
    f(ctx, M.to_device(A), M.to_device(B), C, algo=algo, tile=tile)
    torch.cuda.synchronize()
    return M.to_host(C)


@pytest.mark.parametrize("dist", ["uniform", "illcond"])
def test_skinny_dd_matches_oracle(gpu, dist):
    """64 x 48 x 20037 (a ragged last chunk), default and 32 x 32 tiles,
    every entry within the DD bound."""
    M, ctx = gpu
    m, n, l = 64, 48, 20037
    gen = inputs.dd_uniform if dist == "uniform" else inputs.dd_illcond
    A, B = gen(m, l, 160), gen(l, n, 161)
    for tile in (None, M.variants(2)[1]):
        C = run(M, ctx, A, B, tile)
        r, _ = error_ratio_full(C, A, B, -104)
        print(dist, tile, "ratio", r)
        assert r <= DD_BOUND


@pytest.mark.parametrize("splits", [1, 2, 3, 7, 100, 5000])
def test_explicit_chunk_counts(gpu, splits):
    """Explicit chunk counts, from one chunk (the block kernel) to chunks of a
    single K step; all within the DD bound and bitwise deterministic."""
    M, ctx = gpu
    m, n, l = 70, 50, 3001
    A, B = inputs.dd_illcond(m, l, 162), inputs.dd_illcond(l, n, 163)
    tile = dict(M.variants(2)[7], splits=splits)
    C = run(M, ctx, A, B, tile)
    r, _ = error_ratio_full(C, A, B, -104)
    assert r <= DD_BOUND, (splits, r)
    C2 = run(M, ctx, A, B, tile)
    assert np.array_equal(C[0], C2[0]) and np.array_equal(C[1], C2[1])
    if splits == 1:
        Cb = run(M, ctx, A, B, M.variants(2)[7], "block")
        assert np.array_equal(C[0], Cb[0]) and np.array_equal(C[1], Cb[1])


def test_integer_inputs_bit_exact(gpu):
    """Integer inputs |x| <= 2^30, l = 4096: every partial and every sum of
    partials is exact, so the result is the canonical DD of the integer
    product, bit for bit (DD and QD)."""
    M, ctx = gpu
    m, n, l = 40, 30, 4096
    A, B = inputs.integers(m, l, 2, 164), inputs.integers(l, n, 2, 165)
    Ce = cref.gemm_exact(A, B, out_limbs=2)
    for splits in (0, 5, 16):
        C = run(M, ctx, A, B, {"splits": splits})
        assert np.array_equal(C[0], Ce[0]) and np.array_equal(C[1], Ce[1]), splits
    Aq, Bq = inputs.integers(m, l, 4, 166), inputs.integers(l, n, 4, 167)
    Ceq = cref.gemm_exact(Aq, Bq, out_limbs=4)
    Cq = run(M, ctx, Aq, Bq, {"splits": 0})
    for p, q in zip(Cq, Ceq):
        assert np.array_equal(p, q)


def test_skinny_qd_matches_oracle(gpu):
    M, ctx = gpu
    m, n, l = 33, 31, 8200
    A, B = inputs.qd_uniform(m, l, 168), inputs.qd_uniform(l, n, 169)
    for splits in (0, 9):
        C = run(M, ctx, A, B, {"splits": splits})
        r, _ = error_ratio_full(C, A, B, -208)
        print("QD split-K", splits, "ratio", r)
        assert r <= 8.0


@pytest.mark.parametrize("m,n,l", [(1, 1, 100000), (1, 300, 7000), (2, 2, 512), (5, 3, 1)])
def test_dot_and_thin_shapes(gpu, m, n, l):
    M, ctx = gpu
    A, B = inputs.dd_uniform(m, l, 170), inputs.dd_uniform(l, n, 171)
    C = run(M, ctx, A, B)
    r, _ = error_ratio_full(C, A, B, -104)
    assert r <= DD_BOUND


def test_full_size_skinny_sampled(gpu):
    """64 x 64 x 2^20 (one C tile of the default kernel): both full rows and
    columns at the edges and random entries within the DD bound; equal to a
    second run bit for bit."""
    M, ctx = gpu
    m = n = 64
    l = 1 << 20
    A, B = inputs.dd_uniform(m, l, 172), inputs.dd_uniform(l, n, 173)
    Ad, Bd = M.to_device(A), M.to_device(B)
    C1, C2 = M.empty_like_limbs(m, n, 2), M.empty_like_limbs(m, n, 2)
    M.mpgemm_dd(ctx, Ad, Bd, C1, algo="splitk")
    M.mpgemm_dd(ctx, Ad, Bd, C2, algo="splitk")
    torch.cuda.synchronize()
    assert torch.equal(C1[0], C2[0]) and torch.equal(C1[1], C2[1])
    r = ExactSample(A, B, nrand=64).ratios(M.to_host(C1), -104)
    print("64x64x2^20 split-K max ratio", r.max())
    assert r.max() <= DD_BOUND


def test_auto_table_and_tuner(gpu):
    """MPG_AUTO runs a tabled split-K choice bit for bit; on a skinny shape
    the exhaustive tuner times the split-K candidates and picks one of them
    (the block kernel leaves most of the GPU idle there)."""
    M, ctx = gpu
    T = M.Tuner(ctx)
    m, n, l = 64, 64, 1 << 16
    A, B = inputs.dd_uniform(m, l, 174), inputs.dd_uniform(l, n, 175)
    T.table_set("dd", m, n, l, "splitk", {"splits": 12})
    Ca = run(M, ctx, A, B, None, "auto")
    Cs = run(M, ctx, A, B, {"splits": 12})
    assert np.array_equal(Ca[0], Cs[0]) and np.array_equal(Ca[1], Cs[1])
    r = T.tune("dd", m, n, l, "exhaustive")
    print("skinny tuner pick", r)
    assert r["algo"] == M.MPG_SPLITK
    blk = T.time("dd", m, n, l, "block", None, reps=3)
    assert r["ms"] * 4 < blk
