"""GPU parity of the split-precision (INT8 MFMA) path against the oracle:
digit planes and exponents bit-exact, the integer special case exact, the
value within the recombination tolerance of the oracle's exact truncated
product, and the DD bound against exact AB with the exact slice count."""
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import cref, exact, ozaki
from paper_1710_01839_amd import inputs
from tests.helpers import error_ratio_full, sampled_errors, sampled_pairs

pytestmark = pytest.mark.gpu


def run_oz(M, ctx, A, B, S, mode="all"):
    m, n = A.shape[0], B.shape[1]
    C = M.empty_like_limbs(m, n, 2)
    M.mpgemm_ozaki_dd(ctx, torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda(), C, S, mode)
    torch.cuda.synchronize()
    return M.to_host(C)


@pytest.mark.parametrize("side", [0, 1])
def test_split_planes_bit_exact(gpu, side):
    M, ctx = gpu
    X = inputs.fp64_wide(70, 101, 0)
    S = 12
    planes, exps = M.ozaki_split(ctx, torch.as_tensor(X).cuda(), S, side)
    torch.cuda.synchronize()
    planes, exps = planes.cpu().numpy(), exps.cpu().numpy()
    if side == 0:
        e = ozaki.row_exponents(X)
        D, _ = ozaki.split_rows(X, e, S)
        assert np.array_equal(exps, e)
        for s in range(S):
            assert np.array_equal(planes[s, :70, :101], D[s])
            assert not planes[s, 70:, :].any() and not planes[s, :, 101:].any()
    else:
        f = ozaki.col_exponents(X)
        D, _ = ozaki.split_cols(X, f, S)
        assert np.array_equal(exps, f)
        for s in range(S):
            assert np.array_equal(planes[s, :101, :70], D[s].T)
            assert not planes[s, 101:, :].any() and not planes[s, :, 70:].any()


def _tiny_mix(rows, cols, seed):
    """Normal numbers near 2^-1000 mixed with subnormals, an all-zero row
    and an all-zero column: exercises every branch of the bit-range scan."""
    g = np.random.default_rng(seed)
    X = np.ldexp(g.uniform(0.5, 1.0, (rows, cols)), -1000 - g.integers(0, 40, (rows, cols)))
    sub = g.random((rows, cols)) < 0.2
    X[sub] = np.ldexp(g.integers(1, 2 ** 20, sub.sum()).astype(np.float64), -1074)
    X[g.random((rows, cols)) < 0.5] *= -1
    X[3, :] = 0.0
    X[:, 5] = 0.0
    return X


@pytest.mark.parametrize("kind", ["wide", "subnormal", "uniform"])
def test_slices_exact_matches_oracle(gpu, kind):
    M, ctx = gpu
    if kind == "wide":
        A, B = inputs.fp64_wide(90, 130, 1), inputs.fp64_wide(130, 60, 2)
    elif kind == "subnormal":
        A, B = _tiny_mix(90, 130, 1), _tiny_mix(130, 60, 2)
    else:
        A, B = inputs.dd_uniform(300, 520, 1)[0], inputs.dd_uniform(520, 270, 2)[0]
    At, Bt = torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda()
    S = M.ozaki_slices_exact(ctx, At, Bt)
    assert S == ozaki.slices_exact(A, B)
    for side, X, want in ((0, A, ozaki.row_exponents(A)), (1, B, ozaki.col_exponents(B))):
        _, exps = M.ozaki_split(ctx, torch.as_tensor(X).cuda(), 1, side)
        assert np.array_equal(exps.cpu().numpy(), want), side


def test_single_slice_integer_product_exact(gpu):
    """Integer entries in [-63, 63], row/column maxima >= 32 (scale 2^6, one
    radix-256 digit of weight 1): one digit plane holds them, the MFMA sums
    are exact, C == AB."""
    M, ctx = gpu
    g = np.random.default_rng(3)
    m, n, l = 100, 90, 300
    A = g.integers(-63, 64, size=(m, l)).astype(float)
    B = g.integers(-63, 64, size=(l, n)).astype(float)
    A[:, 5] = 63.0
    B[7, :] = -40.0
    assert ozaki.slices_exact(A, B) == 1
    C = run_oz(M, ctx, A, B, 1)
    want = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(C[0], want.astype(float)) and not C[1].any()


# one case per kernel shape: LDS-staged (1..8), band with two column blocks
# (9..20) and one (21..24), and the general kernel above 24, both pair sets
@pytest.mark.parametrize("S,mode", [(1, "all"), (3, "all"), (7, "all"), (8, "triangle"), (10, "triangle"),
                                    (13, "all"), (20, "all"), (24, "triangle"), (26, "all")])
def test_matches_oracle_truncated_product(gpu, S, mode):
    M, ctx = gpu
    m, n, l = 77, 69, 150
    A, B = inputs.fp64_wide(m, l, 4), inputs.fp64_wide(l, n, 5)
    C = run_oz(M, ctx, A, B, S, mode)
    (hi, lo), (N, E0) = ozaki.ozaki_dd(A, B, S, mode)
    G = cref.absprod_exact((A,), (B,))
    for idx in np.ndindex(hi.shape):
        got = Fraction(float(C[0][idx])) + Fraction(float(C[1][idx]))
        want = ozaki.to_fraction(N, E0, idx)
        # double-double recombination of at most a few hundred exact terms
        assert abs(got - want) <= Fraction(float(G[idx])) * Fraction(256, 2 ** 106) + abs(want) * Fraction(1, 2 ** 104)


def test_exact_slices_meet_dd_bound(gpu):
    """slices = 0 (exact splitting, all pairs): equal stated accuracy with the
    DD kernel, |C - AB| <= 8 l 2^-104 (|A||B|)."""
    M, ctx = gpu
    m, n, l = 128, 96, 257
    A, B = inputs.fp64_wide(m, l, 6), inputs.fp64_wide(l, n, 7)
    C = run_oz(M, ctx, A, B, 0)
    assert M.ozaki_last_slices(ctx) == ozaki.slices_exact(A, B)
    r, _ = error_ratio_full(C, (A,), (B,), -104)
    print("ozaki exact-slices ratio", r, "S =", M.ozaki_last_slices(ctx))
    assert r <= 8.0


@pytest.mark.parametrize("S", [6, 10])
def test_truncated_within_apriori_bound(gpu, S):
    M, ctx = gpu
    m, n, l = 64, 80, 200
    A, B = inputs.fp64_wide(m, l, 8), inputs.fp64_wide(l, n, 9)
    C = run_oz(M, ctx, A, B, S)
    Ce = cref.gemm_exact((A,), (B,), out_limbs=2)
    d = np.abs(cref.exact_diff(C, Ce))
    assert np.all(d <= ozaki.apriori_bound(A, B, S) * (1 + 2.0 ** -40) + np.abs(Ce[0]) * 2.0 ** -100)


def test_edge_cases(gpu):
    M, ctx = gpu
    # zero rows / columns, l not a multiple of 64, 1 x 1
    A = inputs.fp64_wide(33, 65, 10)
    B = inputs.fp64_wide(65, 17, 11)
    A[3, :] = 0.0
    B[:, 4] = 0.0
    C = run_oz(M, ctx, A, B, 0)
    r, _ = error_ratio_full(C, (A,), (B,), -104)
    assert r <= 8.0 and not C[0][3].any() and not C[0][:, 4].any()
    C = run_oz(M, ctx, np.array([[3.0]]), np.array([[-0.5]]), 0)
    assert C[0][0, 0] == -1.5 and C[1][0, 0] == 0.0
    with pytest.raises(M.MpgemmError):
        run_oz(M, ctx, A, B, 41)


def test_full_size_4096_exact_slices_sampled(gpu):
    """n = 4096 (smallest size of the split-precision workload) with the
    exact slice count: DD bound at sampled entries against Python integers."""
    M, ctx = gpu
    n = 4096
    A, B = inputs.fp64_wide(n, n, 12), inputs.fp64_wide(n, n, 13)
    C = run_oz(M, ctx, A, B, 0)
    pairs = sampled_pairs(n, n, 32)
    errs, mags = sampled_errors(C, (A,), (B,), pairs)
    r = max(e / (n * 2.0 ** -104 * g) for e, g in zip(errs, mags) if g > 0)
    print("n=4096 exact slices", M.ozaki_last_slices(ctx), "ratio", r)
    assert r <= 8.0


def run_ddoz(M, ctx, A, B, S, mode="all"):
    m, n = A[0].shape[0], B[0].shape[1]
    C = M.empty_like_limbs(m, n, 2)
    M.mpgemm_dd_ozaki(ctx, M.to_device(A), M.to_device(B), C, S, mode)
    torch.cuda.synchronize()
    return M.to_host(C)


@pytest.mark.parametrize("dist", ["uniform", "illcond"])
def test_dd_inputs_exact_slices(gpu, dist):
    """Double-double inputs with the exact slice count: the count is the
    oracle's, C meets the DD bound against the exact product of the limb
    sums, and mpgemm_dd(algo='ozaki') gives the same bits."""
    M, ctx = gpu
    gen = inputs.dd_uniform if dist == "uniform" else inputs.dd_illcond
    m, n, l = 96, 80, 203
    A, B = gen(m, l, 20), gen(l, n, 21)
    C = run_ddoz(M, ctx, A, B, 0)
    S = M.ozaki_last_slices(ctx)
    assert S == ozaki.slices_exact(A, B)
    r, _ = error_ratio_full(C, A, B, -104)
    print(dist, "DD-input exact slices", S, "ratio", r)
    assert r <= 8.0
    C2 = M.empty_like_limbs(m, n, 2)
    M.mpgemm_dd(ctx, M.to_device(A), M.to_device(B), C2, algo="ozaki", tile={"slices": 0})
    torch.cuda.synchronize()
    C2 = M.to_host(C2)
    assert np.array_equal(C[0], C2[0]) and np.array_equal(C[1], C2[1])


@pytest.mark.parametrize("S,mode", [(5, "all"), (9, "triangle"), (12, "all")])
def test_dd_inputs_match_oracle_truncated(gpu, S, mode):
    """Truncated slicing of double-double inputs: the value the oracle's
    two-limb split gives, up to the double-double recombination (a digit
    taken differently would move C by far more)."""
    M, ctx = gpu
    m, n, l = 40, 36, 70
    A, B = inputs.dd_uniform(m, l, 22), inputs.dd_uniform(l, n, 23)
    C = run_ddoz(M, ctx, A, B, S, mode)
    (hi, lo), (N, E0) = ozaki.ozaki_dd(A, B, S, mode)
    G = cref.absprod_exact(A, B)
    for idx in np.ndindex(hi.shape):
        got = Fraction(float(C[0][idx])) + Fraction(float(C[1][idx]))
        want = ozaki.to_fraction(N, E0, idx)
        assert abs(got - want) <= Fraction(float(G[idx])) * Fraction(256, 2 ** 106) + abs(want) * Fraction(1, 2 ** 104)


@pytest.mark.parametrize("S", [0, 6])
def test_dd_inputs_zero_lo_reduce_to_fp64_path(gpu, S):
    """lo = 0: the two-limb split takes the same digits as the FP64 split,
    so both entry points return the same bits (and slice count)."""
    M, ctx = gpu
    m, n, l = 70, 130, 190
    A, B = inputs.fp64_wide(m, l, 25), inputs.fp64_wide(l, n, 26)
    C1 = run_oz(M, ctx, A, B, S)
    S1 = M.ozaki_last_slices(ctx)
    C2 = run_ddoz(M, ctx, (A, np.zeros_like(A)), (B, np.zeros_like(B)), S)
    assert M.ozaki_last_slices(ctx) == S1
    assert np.array_equal(C1[0], C2[0]) and np.array_equal(C1[1], C2[1])


@pytest.mark.parametrize("bits", [40, 106])
def test_slice_tuner_meets_target(gpu, bits):
    """The slice count and pair set the tuner picks for a target of `bits`
    meet |C - AB|_ij <= l 2^(e_i + f_j) 2^-bits (plus the DD rounding of the
    recombination) against the exact product."""
    M, ctx = gpu
    m, n, l = 96, 80, 300
    A, B = inputs.fp64_wide(m, l, 12), inputs.fp64_wide(l, n, 13)
    r = M.Tuner(ctx).tune_slices(m, n, l, bits)
    print("bits", bits, r)
    assert r["slices"] == ozaki.slices_for_bits(bits, r["pairs"]) and r["ms"] > 0
    C = run_oz(M, ctx, A, B, r["slices"], r["pairs"])
    Ce = cref.gemm_exact((A,), (B,), out_limbs=2)
    d = np.abs(cref.exact_diff(C, Ce))
    e, f = ozaki.row_exponents(A), ozaki.col_exponents(B)
    target = l * np.ldexp(1.0, (e[:, None] + f[None, :]).astype(np.int64)) * 2.0 ** -bits
    assert np.all(d <= target * (1 + 2.0 ** -40) + np.abs(Ce[0]) * 2.0 ** -100)


def test_slice_tuner_exact_count_competes(gpu):
    """With the data given, the exact slice count (7 for uniform [-1, 1)
    data) replaces the all-pairs count of a 106-bit target (14)."""
    M, ctx = gpu
    n = 512
    A, B = inputs.dd_uniform(n, n, 3)[0], inputs.dd_uniform(n, n, 4)[0]
    S_exact = ozaki.slices_exact(A, B)
    r = M.Tuner(ctx).tune_slices(n, n, n, 106, torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda())
    print("exact", S_exact, r)
    assert (r["pairs"], r["slices"]) in {("all", S_exact), ("triangle", ozaki.slices_for_bits(106, "triangle"))}
    with pytest.raises(M.MpgemmError):
        M.Tuner(ctx).tune_slices(n, n, n, 0)
    with pytest.raises(M.MpgemmError):
        M.Tuner(ctx).tune_slices(n, n, n, 400)     # beyond 40 slices


def test_dd_inputs_carry_patterns(gpu):
    """Elements just inside a power of two, of both signs, have digit
    expansions that are long runs of 255 and carry from the lowest digit
    into the top one.  Double-double inputs (power-of-two hi, lo of the
    opposite sign) with the exact slice count give the exact product up to
    the recombination; FP64 inputs with all-ones mantissas split into the
    oracle's digit planes bit for bit."""
    M, ctx = gpu
    g = np.random.default_rng(9)
    m, n, l = 40, 36, 70
    sign = np.where(g.random((m, l)) < 0.5, -1.0, 1.0)
    hi = sign * np.ldexp(1.0, g.integers(-6, 1, (m, l)) - 1)
    lo = -sign * np.ldexp(np.abs(hi), -53 - g.integers(1, 20, (m, l)))
    A, B = (hi, lo), inputs.dd_uniform(l, n, 10)
    Ct = run_ddoz(M, ctx, A, B, 0)
    S = M.ozaki_last_slices(ctx)
    assert S == ozaki.slices_exact(A, B)
    r, _ = error_ratio_full(Ct, A, B, -104)
    print("carry patterns: exact slices", S, "ratio", r)
    assert r <= 8.0
    X = sign * (np.ldexp(1.0, g.integers(-6, 1, (m, l))) * (1.0 - 2.0 ** -53))
    planes, exps = M.ozaki_split(ctx, torch.as_tensor(X).cuda(), 9, 0)
    torch.cuda.synchronize()
    D, _ = ozaki.split_rows(X, ozaki.row_exponents(X), 9)
    assert any(int(d.min()) < 0 for d in D[1:]) and any(int(d.max()) > 0 for d in D[1:])
    for s_ in range(9):
        assert np.array_equal(planes.cpu().numpy()[s_, :m, :l], D[s_])


# K longer than one INT32 chunk (2048 / S steps of 64): the double-double
# partial results wait in C between chunks.  One case per kernel family,
# and K = 32704 (the general kernel's limit, here with 7 slices).
@pytest.mark.parametrize("kind,l", [("uniform", 20480), ("dd", 8192), ("wide", 8192), ("uniform", 32704)])
def test_multi_chunk_k(gpu, kind, l):
    M, ctx = gpu
    m, n = 48, 40
    if kind == "dd":
        A, B = inputs.dd_uniform(m, l, 21), inputs.dd_uniform(l, n, 22)
        C = run_ddoz(M, ctx, A, B, 0)
    else:
        gen = inputs.fp64_wide if kind == "wide" else (lambda r, c, s: inputs.dd_uniform(r, c, s)[0])
        A, B = (gen(m, l, 21),), (gen(l, n, 22),)
        C = run_oz(M, ctx, A[0], B[0], 0)
    S = M.ozaki_last_slices(ctx)
    assert (l // 64) > 2048 // S                    # more than one chunk
    r, _ = error_ratio_full(C, A, B, -104, threads=8)
    print(kind, "l", l, "slices", S, "chunks", -(-(l // 64) // (2048 // S)), "ratio", r)
    assert r <= 8.0


def test_k_beyond_headroom_refused(gpu):
    """Up to 24 slices K is cut into INT32-safe chunks, so any l works (all
    ones: C = l exactly); above 24 slices the general kernel keeps each
    diagonal sum over the whole of K, and l > 32704 is refused."""
    M, ctx = gpu
    l = 40000
    A = torch.ones(4, l, dtype=torch.float64, device="cuda")
    B = torch.ones(l, 4, dtype=torch.float64, device="cuda")
    C = M.empty_like_limbs(4, 4, 2)
    M.mpgemm_ozaki_dd(ctx, A, B, C, 0)
    torch.cuda.synchronize()
    assert torch.all(C[0] == float(l)) and torch.all(C[1] == 0.0)
    A[:, 1] = 2.0 ** -200                       # 26 slices for these rows
    assert M.ozaki_slices_exact(ctx, A, B) > 24
    with pytest.raises(M.MpgemmError):
        M.mpgemm_ozaki_dd(ctx, A, B, C, 0)


def test_int8_mfma_rate(gpu):
    """The sustained INT8 matrix-core rate the split products are compared
    with: positive and below the datasheet's dense peak (5.0 POP/s) with a
    margin for clock boost."""
    M, ctx = gpu
    tops = M.int8_mfma_rate(ctx)
    print("sustained INT8 MFMA rate", tops, "TOP/s")
    assert 1000.0 < tops < 5600.0
