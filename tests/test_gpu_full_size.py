"""Parity at the configurations' full sizes and on ragged multi-tile shapes.

* DD block kernel at n = 4096 (uniform and ill-conditioned inputs) and at
  n = 1024, 2048: two full rows, two full columns and random entries
  against the oracle's exact product, componentwise bound
  8 l 2^-104 (|A||B|)_ij.
* Strassen (Winograd's form): the GPU's normwise error stays within a small
  factor of the oracle's own step-by-step Winograd recursion of the same
  depth on the same inputs (and within Higham's bound).
* The split product at n = 8192 (digit and residue forms, exact slice
  count, the wide FP64 workload and the DD workload), the residue form on
  the wide workload at n = 4096, and every entry of a ragged shape that
  spans several 256 x 256 residue-product tiles and K steps.
* Truncated slice counts S = 6..10 on the split-precision workload at
  n = 4096 and 8192: measured componentwise and normwise errors per S,
  within the a-priori truncation bound.
"""
import numpy as np
import pytest
import torch

from oracle import cref, crt, ozaki
from paper_1710_01839_amd import inputs
from tests.helpers import ExactSample, error_ratio_full, winograd_bound

pytestmark = pytest.mark.gpu

DD_BOUND = 8.0            # |C - AB| <= 8 l 2^-104 (|A||B|)


def _dd(M, ctx, A, B, algo="block", tile=None):
    m, n = A[0].shape[0], B[0].shape[1]
    C = M.empty_like_limbs(m, n, 2)
    M.mpgemm_dd(ctx, M.to_device(A), M.to_device(B), C, algo=algo, tile=tile)
    torch.cuda.synchronize()
    return M.to_host(C)


def _split(M, ctx, A, B, S, mode):
    """A, B: FP64 arrays or (hi, lo) tuples; mode 'all' (digit form) or 'crt'."""
    dd = isinstance(A, tuple)
    m, n = (A[0] if dd else A).shape[0], (B[0] if dd else B).shape[1]
    C = M.empty_like_limbs(m, n, 2)
    if dd:
        M.mpgemm_dd_ozaki(ctx, M.to_device(A), M.to_device(B), C, S, mode)
    else:
        M.mpgemm_ozaki_dd(ctx, torch.as_tensor(A).cuda(), torch.as_tensor(B).cuda(), C, S, mode)
    torch.cuda.synchronize()
    return M.to_host(C)


# ---------------------------------------------------------------------------
# double-double kernels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dist", ["uniform", "illcond"])
def test_dd_block_4096_rows_cols_random(gpu, dist):
    """n = 4096 block kernel (the default, load-unit-staged tile): rows 0 and
    n-1, columns 0 and n-1 and 1024 random entries against the exact product;
    ill-conditioned inputs with hi = U[-1,1] 2^k, k ~ U{-30..30}."""
    M, ctx = gpu
    n = 4096
    gen = inputs.dd_uniform if dist == "uniform" else inputs.dd_illcond
    A, B = gen(n, n, 130), gen(n, n, 131)
    C = _dd(M, ctx, A, B)
    r = ExactSample(A, B, nrand=1024).ratios(C, -104)
    print(f"n=4096 block {dist}: max componentwise ratio {r.max():.4g} over {r.size} entries")
    assert r.max() <= DD_BOUND


@pytest.mark.parametrize("n", [1024, 2048])
def test_dd_block_smaller_sizes(gpu, n):
    """The configuration's n = 1024 and 2048 with the default tile and with the
    register-staged 64 x 64 x 16 tile."""
    M, ctx = gpu
    A, B = inputs.dd_illcond(n, n, 132), inputs.dd_illcond(n, n, 133)
    sample = ExactSample(A, B, nrand=512)
    for tile in (None, M.variants(2)[0]):
        r = sample.ratios(_dd(M, ctx, A, B, "block", tile), -104)
        print(f"n={n} block {tile}: max ratio {r.max():.4g}")
        assert r.max() <= DD_BOUND


_STRASSEN_CACHE = {}


def _strassen_operands(n):
    return inputs.dd_uniform(n, n, 134), inputs.dd_uniform(n, n, 135)


def _strassen_exact(n):
    if n not in _STRASSEN_CACHE:
        _STRASSEN_CACHE[n] = cref.gemm_exact(*_strassen_operands(n), out_limbs=3)
    return _STRASSEN_CACHE[n]


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_strassen_error_tracks_oracle_recursion(gpu, depth):
    """Winograd's recursion on the GPU against the oracle's step-by-step
    Winograd recursion of the same depth (accurate DD operations): the
    GPU's normwise error is within a factor 16 of the oracle's (a dropped
    term or a wrong sign in an operand or assembly sum would be many orders
    larger) and within Higham's bound."""
    M, ctx = gpu
    n = 512
    A, B = _strassen_operands(n)
    Ce = _strassen_exact(n)
    amax, bmax = float(np.abs(A[0]).max()) * (1 + 2.0 ** -50), float(np.abs(B[0]).max()) * (1 + 2.0 ** -50)

    def normwise(C):
        d = np.abs(cref.exact_diff(C, Ce)) * (1 + 2.0 ** -52) + np.abs(Ce[0]) * 2.0 ** -160
        return float(d.max() / (amax * bmax))

    r_gpu = normwise(_dd(M, ctx, A, B, "strassen", {"depth": depth}))
    r_orc = normwise(cref.gemm_strassen(A, B, depth, "winograd"))
    r_blk = normwise(_dd(M, ctx, A, B, "block"))
    bound = winograd_bound(n, depth, 8 * 2.0 ** -104)
    print(f"depth {depth}: gpu {r_gpu:.3g} oracle winograd {r_orc:.3g} block {r_blk:.3g} bound {bound:.3g}")
    assert r_gpu <= 16 * r_orc
    assert r_gpu <= bound


# ---------------------------------------------------------------------------
# split product at full size
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("workload,mode", [("wide", "all"), ("wide", "crt"), ("dd", "all"), ("dd", "crt")])
def test_split_8192_exact_slices(gpu, workload, mode):
    """n = 8192 with the exact slice count: digit form (all pairs) and
    residue form, FP64 inputs U[-1,1] 2^round(N(0,10)) and DD inputs; the DD
    bound at sampled rows, columns and random entries, and for the residue
    form the single rounding of the exact product (2^-104 relative)."""
    M, ctx = gpu
    n = 8192
    if workload == "wide":
        Ah, Bh = inputs.fp64_wide(n, n, 136), inputs.fp64_wide(n, n, 137)
        A, B = (Ah,), (Bh,)
        C = _split(M, ctx, Ah, Bh, 0, mode)
    else:
        A, B = inputs.dd_uniform(n, n, 138), inputs.dd_uniform(n, n, 139)
        C = _split(M, ctx, A, B, 0, mode)
    S = M.ozaki_last_slices(ctx)
    sample = ExactSample(A, B, nrand=256)
    r = sample.ratios(C, -104)
    rel = sample.errors(C) / np.where(sample.Ce[0] != 0, np.abs(sample.Ce[0]), np.inf)
    print(f"n=8192 {workload} {mode}: slices {S}, moduli {M.ozaki_last_moduli(ctx)}, "
          f"max ratio {r.max():.4g}, max |C-AB|/|AB| {rel.max():.4g}")
    assert r.max() <= DD_BOUND
    if mode == "crt":
        assert rel.max() <= 2.0 ** -104 * (1 + 2.0 ** -40)


def test_residue_form_wide_4096(gpu):
    """The residue form on the wide FP64 workload at n = 4096 (the bench's
    configuration): one rounding of the exact product."""
    M, ctx = gpu
    n = 4096
    A, B = inputs.fp64_wide(n, n, 140), inputs.fp64_wide(n, n, 141)
    C = _split(M, ctx, A, B, 0, "crt")
    sample = ExactSample((A,), (B,), nrand=1024)
    rel = sample.errors(C) / np.where(sample.Ce[0] != 0, np.abs(sample.Ce[0]), np.inf)
    print(f"n=4096 wide residue form: slices {M.ozaki_last_slices(ctx)}, moduli {M.ozaki_last_moduli(ctx)}, "
          f"max |C-AB|/|AB| {rel.max():.4g}")
    assert rel.max() <= 2.0 ** -104 * (1 + 2.0 ** -40)
    assert np.all(sample.ratios(C, -104) <= DD_BOUND)


# ---------------------------------------------------------------------------
# residue form on a ragged shape of several tiles, every entry
# ---------------------------------------------------------------------------

SHAPE = (600, 520, 333)   # 3 x 3 tiles of 256 x 256 (ragged), 6 K steps of 64 (ragged)


@pytest.mark.parametrize("kind", ["dd", "wide", "uniform"])
def test_residue_multitile_exact(gpu, kind):
    """Exact slice count: every entry is the exact product rounded once to
    double-double (|C - AB| <= 2^-104 |AB|)."""
    M, ctx = gpu
    m, n, l = SHAPE
    if kind == "dd":
        A, B = inputs.dd_illcond(m, l, 142, kmax=12), inputs.dd_illcond(l, n, 143, kmax=12)
        C = _split(M, ctx, A, B, 0, "crt")
    else:
        gen = inputs.fp64_wide if kind == "wide" else (lambda r, c, s: inputs.dd_uniform(r, c, s)[0])
        Ah, Bh = gen(m, l, 144), gen(l, n, 145)
        A, B = (Ah,), (Bh,)
        C = _split(M, ctx, Ah, Bh, 0, "crt")
    assert M.ozaki_last_slices(ctx) == ozaki.slices_exact(A, B)
    Ce = cref.gemm_exact(A, B, out_limbs=3)
    d = np.abs(cref.exact_diff(C, Ce)) * (1 + 2.0 ** -52) + np.abs(Ce[0]) * 2.0 ** -160
    assert np.all(d <= 2.0 ** -104 * np.abs(Ce[0]) * (1 + 2.0 ** -40))
    print(kind, "slices", M.ozaki_last_slices(ctx), "moduli", M.ozaki_last_moduli(ctx),
          "max |C-AB| / (2^-104 |AB|)", float(np.max(np.where(Ce[0] != 0, d / (2.0 ** -104 * np.abs(Ce[0])), 0))))


def test_residue_multitile_truncated(gpu):
    """Five slices (fewer than exact): every entry is the exact product of the
    truncated integer images X = A' B' scaled by 2^(e_i + f_j + 4 - 16 S),
    rounded once.  Images of five slices are below 2^38, so the oracle forms
    X exactly with its super-accumulator from the images as doubles."""
    M, ctx = gpu
    m, n, l = SHAPE
    S = 5
    A, B = inputs.dd_uniform(m, l, 146), inputs.dd_uniform(l, n, 147)
    C = _split(M, ctx, A, B, S, "crt")
    e, f = ozaki.row_exponents(A[0]), ozaki.col_exponents(B[0])
    IA = crt.images_rows(A, e, S).astype(np.float64)
    IB = crt.images_cols(B, f, S).astype(np.float64)
    assert np.abs(IA).max() < 2.0 ** 38 and np.abs(IB).max() < 2.0 ** 38
    X = cref.gemm_exact((np.ascontiguousarray(IA),), (np.ascontiguousarray(IB),), out_limbs=3)
    sc = (e[:, None] + f[None, :] + 4 - 16 * S).astype(np.int64)
    V = tuple(np.ldexp(x, sc) for x in X)            # exact: powers of two, no underflow here
    d = np.abs(cref.exact_diff(C, V)) * (1 + 2.0 ** -52) + np.abs(V[0]) * 2.0 ** -160
    assert np.all(d <= 2.0 ** -104 * np.abs(V[0]) * (1 + 2.0 ** -40))


def test_qd_residue_multitile(gpu):
    """Quad-double through the residue form on the ragged multi-tile shape:
    every entry within the QD kernels' bound 8 l 2^-208 (|A||B|)_ij."""
    M, ctx = gpu
    m, n, l = SHAPE
    A, B = inputs.qd_uniform(m, l, 148), inputs.qd_uniform(l, n, 149)
    C = M.empty_like_limbs(m, n, 4)
    M.mpgemm_qd(ctx, M.to_device(A), M.to_device(B), C, algo="ozaki_crt")
    torch.cuda.synchronize()
    r, _ = error_ratio_full(M.to_host(C), A, B, -208)
    print("QD residue form multi-tile ratio", r)
    assert r <= 8.0


# ---------------------------------------------------------------------------
# truncated slice counts of the configuration (6..10 slices)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [4096, 8192])
def test_truncated_slices_error_per_count(gpu, n):
    """S = 6..10 slices on U[-1,1] 2^round(N(0,10)): for the digit form (all
    pairs) and the residue form, the measured error at sampled entries,
    componentwise (|C - AB| / (|A||B|)) and normwise (|C - AB| / (max|A|
    max|B|)), each entry within the a-priori truncation bound
    l 2^(e_i + f_j) 2^(3 - 8S) plus the recombination (digit form) or the
    final rounding (residue form); the errors fall with S."""
    M, ctx = gpu
    A, B = inputs.fp64_wide(n, n, 150), inputs.fp64_wide(n, n, 151)
    sample = ExactSample((A,), (B,), nrand=256)
    e, f = ozaki.row_exponents(A), ozaki.col_exponents(B)
    scale = n * np.ldexp(1.0, (e[sample.I] + f[sample.J]).astype(np.int64))
    amax, bmax = float(np.abs(A).max()), float(np.abs(B).max())
    absAB = np.abs(sample.Ce[0])
    print(f"\nn={n}: S, form, max |C-AB|/(|A||B|), max |C-AB|/(max|A| max|B|), "
          f"max |C-AB|/(l 2^(e+f)), a-priori 2^(3-8S)")
    prev = {}
    for S in range(6, 11):
        for mode in ("all", "crt"):
            C = _split(M, ctx, A, B, S, mode)
            err = sample.errors(C)
            comp = float(np.max(np.where(sample.G > 0, err / sample.G, 0.0)))
            norm = float(err.max() / (amax * bmax))
            unit = float(np.max(err / scale))
            apriori = ozaki.apriori_unit(S, "all")
            print(f"  {S:2d} {'digit' if mode == 'all' else 'residue':7s} {comp:.3e} {norm:.3e} {unit:.3e} "
                  f"{apriori:.3e}")
            round_slack = (2.0 ** -100 if mode == "all" else 2.0 ** -104) * absAB
            assert np.all(err <= scale * apriori * (1 + 2.0 ** -40) + round_slack)
            if mode in prev:
                assert norm < prev[mode]
            prev[mode] = norm
