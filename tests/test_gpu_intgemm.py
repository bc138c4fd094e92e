"""GPU parity of the exact long-integer (fixed-point) product against the
exact oracle: every word of every entry equal (bit-exact), for operand sizes
from 32 to 2048 bits, signs and extreme values, ragged shapes, long K, and
the argument checks."""
import numpy as np
import pytest
import torch

from oracle import bigint

pytestmark = pytest.mark.gpu


def rand_planes(g, rows, cols, words, extreme=False):
    """Uniform two's complement integers of 32 words bits (every bit random);
    with extreme, the most negative and most positive values mixed in."""
    P = g.integers(0, 1 << 32, size=(words, rows, cols), dtype=np.uint64).astype(np.uint32)
    if extreme:
        P[:, 0, :] = 0
        P[-1, 0, :] = 0x80000000          # most negative
        P[:, -1, :] = 0xFFFFFFFF
        P[-1, -1, :] = 0x7FFFFFFF         # most positive
    return P


def run(M, ctx, A, B, words_c=None):
    l = A.shape[2]
    wc = words_c or M.int_words_needed(A.shape[0], B.shape[0], l)
    Ad = torch.as_tensor(A.view(np.int32)).cuda()
    Bd = torch.as_tensor(B.view(np.int32)).cuda()
    Cd = torch.empty((wc, A.shape[1], B.shape[2]), dtype=torch.int32, device="cuda")
    M.int_gemm(ctx, Ad, Bd, Cd)
    torch.cuda.synchronize()
    return Cd.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("wa,wb", [(1, 1), (2, 3), (4, 4), (5, 9), (8, 8), (16, 16), (32, 7)])
def test_bit_exact(gpu, wa, wb):
    M, ctx = gpu
    g = np.random.default_rng(wa * 100 + wb)
    m, n, l = 67, 45, 83
    A = rand_planes(g, m, l, wa, extreme=True)
    B = rand_planes(g, l, n, wb, extreme=True)
    C = run(M, ctx, A, B)
    want = bigint.gemm(A, B)
    print(wa, wb, "words_c", C.shape[0], "moduli", M._lib.mpg_ozaki_last_moduli(ctx.handle))
    assert np.array_equal(C, want)


def test_2048_bits_and_small_values(gpu):
    """64-word operands (2048 bits, 16 chunks: 31 diagonals, up to 16 chunk
    pairs per product); then small values in wide words (upper chunks zero or
    sign extension)."""
    M, ctx = gpu
    g = np.random.default_rng(7)
    A = rand_planes(g, 9, 20, 64)
    B = rand_planes(g, 20, 11, 64)
    assert np.array_equal(run(M, ctx, A, B), bigint.gemm(A, B))
    small_a = np.zeros((12, 30, 40), dtype=np.uint32)
    small_b = np.zeros((12, 40, 20), dtype=np.uint32)
    va = g.integers(-1000, 1000, size=(30, 40))
    vb = g.integers(-1000, 1000, size=(40, 20))
    small_a[:] = np.where(va < 0, 0xFFFFFFFF, 0).astype(np.uint32)
    small_b[:] = np.where(vb < 0, 0xFFFFFFFF, 0).astype(np.uint32)
    small_a[0] = va.astype(np.int64).astype(np.uint32)
    small_b[0] = vb.astype(np.int64).astype(np.uint32)
    C = run(M, ctx, small_a, small_b)
    assert np.array_equal(C, bigint.gemm(small_a, small_b))


def test_long_k(gpu):
    """l = 9000: several reductions of the INT32 sums inside each product."""
    M, ctx = gpu
    g = np.random.default_rng(8)
    A = rand_planes(g, 5, 9000, 4)
    B = rand_planes(g, 9000, 6, 2)
    assert np.array_equal(run(M, ctx, A, B), bigint.gemm(A, B))


def test_full_size_sampled(gpu):
    """m = n = l = 1024 with 1024-bit operands: sampled entries exact."""
    M, ctx = gpu
    g = np.random.default_rng(9)
    nn, w = 1024, 32
    A = rand_planes(g, nn, nn, w)
    B = rand_planes(g, nn, nn, w)
    C = run(M, ctx, A, B)
    rows = [0, 5, 511, nn - 1]
    cols = [0, 17, 700, nn - 1]
    want = bigint.gemm(np.ascontiguousarray(A[:, rows, :]), np.ascontiguousarray(B[:, :, cols]), C.shape[0])
    assert np.array_equal(C[:, rows][:, :, cols], want)


def test_argument_checks(gpu):
    M, ctx = gpu
    A = torch.zeros((2, 4, 4), dtype=torch.int32, device="cuda")
    B = torch.zeros((2, 4, 4), dtype=torch.int32, device="cuda")
    small = torch.zeros((4, 4, 4), dtype=torch.int32, device="cuda")   # needs 5 words
    assert M.int_words_needed(2, 2, 4) == 5
    with pytest.raises(M.MpgemmError) as ei:
        M.int_gemm(ctx, A, B, small)
    assert ei.value.status == M.MPG_ERR_ARG
    with pytest.raises(M.MpgemmError):
        M.int_gemm(ctx, torch.zeros((65, 4, 4), dtype=torch.int32, device="cuda"), B,
                   torch.zeros((70, 4, 4), dtype=torch.int32, device="cuda"))
    C = torch.full((5, 4, 4), 7, dtype=torch.int32, device="cuda")
    M.int_gemm(ctx, A, B, C)       # zero operands: C := 0 in every word
    torch.cuda.synchronize()
    assert not C.any()


def test_empty_inner_dimension_and_alias(gpu):
    """l = 0: every word of C := 0 (the empty sum).  C overlapping an input:
    MPG_ERR_ALIAS, refused before any launch, C unchanged."""
    M, ctx = gpu
    A = torch.zeros((3, 5, 0), dtype=torch.int32, device="cuda")
    B = torch.zeros((2, 0, 6), dtype=torch.int32, device="cuda")
    wc = M.int_words_needed(3, 2, 0)
    assert wc == bigint.words_needed(3, 2, 0)
    C = torch.full((wc, 5, 6), -1, dtype=torch.int32, device="cuda")
    M.int_gemm(ctx, A, B, C)
    torch.cuda.synchronize()
    assert not C.any()

    buf = torch.arange(200, dtype=torch.int32, device="cuda")
    A2 = buf[0:32].view(2, 4, 4)
    C2 = buf[16:96].view(5, 4, 4)            # shares buf[16:32] with A2
    B2 = torch.ones((2, 4, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(M.MpgemmError) as ei:
        M.int_gemm(ctx, A2, B2, C2)
    assert ei.value.status == M.MPG_ERR_ALIAS
    torch.cuda.synchronize()
    assert torch.equal(buf, torch.arange(200, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("wa,wb,m,n,l", [(64, 64, 9, 11, 20), (16, 16, 40, 33, 300), (5, 9, 30, 21, 70),
                                          (32, 7, 12, 10, 40), (3, 3, 70, 66, 130)])
def test_every_plan_bit_exact(gpu, wa, wb, m, n, l):
    """Every candidate plan (chunks of 96, 128, 160 bits; Karatsuba depth
    0..2) and, for 64-word operands, depth 3 (sums of eight chunks) gives
    the exact product, word for word; extreme values included."""
    M, ctx = gpu
    g = np.random.default_rng(wa * 1000 + wb * 10 + 3)
    A = rand_planes(g, m, l, wa, extreme=True)
    B = rand_planes(g, l, n, wb, extreme=True)
    want = bigint.gemm(A, B)
    plans = M.int_candidates(wa, wb, l)
    assert plans
    if wa == 64:
        plans = plans + [{"chunk_words": 4, "karatsuba_depth": 3}]
    wc = M.int_words_needed(wa, wb, l)
    Ad = torch.as_tensor(A.view(np.int32)).cuda()
    Bd = torch.as_tensor(B.view(np.int32)).cuda()
    for plan in plans:
        Cd = torch.full((wc, m, n), -1, dtype=torch.int32, device="cuda")
        M.int_gemm(ctx, Ad, Bd, Cd, plan)
        torch.cuda.synchronize()
        got = Cd.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), plan


def test_plan_limits(gpu):
    """A plan that does not fit is refused before anything runs: 96-bit chunks
    of 64-word operands without splitting (22 chunk pairs on a diagonal, more
    than the 16 segments of one product), a depth whose sums exceed eight
    chunks, an unknown chunk width."""
    M, ctx = gpu
    A = torch.zeros((64, 2, 3), dtype=torch.int32, device="cuda")
    B = torch.zeros((64, 3, 2), dtype=torch.int32, device="cuda")
    C = torch.zeros((M.int_words_needed(64, 64, 3), 2, 2), dtype=torch.int32, device="cuda")
    for plan in ({"chunk_words": 3, "karatsuba_depth": 0}, {"chunk_words": 4, "karatsuba_depth": 4},
                 {"chunk_words": 6, "karatsuba_depth": 0}):
        with pytest.raises(M.MpgemmError) as ei:
            M.int_gemm(ctx, A, B, C, plan)
        assert ei.value.status == M.MPG_ERR_UNSUPPORTED, plan


def test_int_tuner_modes_and_table(gpu, tmp_path):
    """The three tuning modes on a 2048-bit product; the paper's procedure
    times at most two plans at full size; MLP mode (trained on exhaustive
    timings of other shapes) times one plan per four; the winner enters the
    table mpg_int_gemm uses (bit for bit the explicit plan's result)."""
    M, ctx = gpu
    T = M.Tuner(ctx)
    db = str(tmp_path / "int.jsonl")
    T.set_db(db)
    for shape in ((256, 256, 256, 64, 64), (512, 256, 512, 32, 32), (256, 512, 1024, 16, 16),
                  (512, 512, 256, 64, 64)):
        T.int_tune(*shape, "exhaustive")
    T.set_db(None)
    mlp = M.MLP(ctx)
    loss, rows = mlp.train_db(db, 2000, 3e-3)
    assert rows >= 20
    shape = (384, 384, 512, 64, 64)
    ncand = len(M.int_candidates(64, 64, 512))
    ex = T.int_tune(*shape, "exhaustive")
    pa = T.int_tune(*shape, "paper")
    ml = T.int_tune(*shape, "mlp")
    print("int tuning", ex, pa, ml)
    assert ex["trials"] == ncand and pa["trials"] <= 2 and ml["trials"] == max(2, (ncand + 3) // 4)
    g = np.random.default_rng(9)
    A = rand_planes(g, 384, 512, 64)
    B = rand_planes(g, 512, 384, 64)
    Ad = torch.as_tensor(A.view(np.int32)).cuda()
    Bd = torch.as_tensor(B.view(np.int32)).cuda()
    wc = M.int_words_needed(64, 64, 512)
    C1 = torch.empty((wc, 384, 384), dtype=torch.int32, device="cuda")
    C2 = torch.empty_like(C1)
    M.int_gemm(ctx, Ad, Bd, C1)                     # the table's plan (MLP mode ran last)
    M.int_gemm(ctx, Ad, Bd, C2, ml["algo"])
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    assert np.array_equal(C1.cpu().numpy().view(np.uint32), bigint.gemm(A, B))


def test_int_slab_prediction(gpu):
    """Section 3's prediction for the long-integer product (slabs of one and
    two waves of the residue products, extrapolated in tile rows) is within
    10% of the measured full-size time, and the slabs cost less than the
    product."""
    M, ctx = gpu
    T = M.Tuner(ctx)
    shape = (4096, 512, 512, 64, 64)
    for plan in ({"chunk_words": 4, "karatsuba_depth": 0}, {"chunk_words": 4, "karatsuba_depth": 2},
                 {"chunk_words": 5, "karatsuba_depth": 1}):
        real = T.int_time(*shape, plan, reps=3)
        pred, slab = T.int_predict(*shape, plan)
        print("int prediction", plan, "predicted %.3f slabs %.3f real %.3f error %.1f%%"
              % (pred, slab, real, 100 * abs(pred - real) / real))
        assert abs(pred - real) <= 0.10 * real
        assert slab < real
