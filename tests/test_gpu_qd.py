"""GPU parity of the quad-double path against the oracle: componentwise bound
8 l 2^-208 (|A||B|)_ij for simple and block, normwise Winograd bound for
Strassen, integer inputs exact."""
import numpy as np
import pytest
import torch

from oracle import cref
from paper_1710_01839_amd import inputs
from tests.helpers import (error_ratio_exact_python, error_ratio_full, normwise_ratio,
                           sampled_errors, sampled_pairs, winograd_bound)

pytestmark = pytest.mark.gpu

QD_BOUND = 8.0            # |C - AB| <= 8 l 2^-208 (|A||B|)
QD_UNIT = 8 * 2.0 ** -208


def run_qd(M, ctx, A, B, algo="block", tile=None):
    m, n = A[0].shape[0], B[0].shape[1]
    C = M.empty_like_limbs(m, n, 4)
    M.mpgemm_qd(ctx, M.to_device(A), M.to_device(B), C, algo=algo, tile=tile)
    torch.cuda.synchronize()
    return M.to_host(C)


def test_qd_simple_small_exact_python(gpu):
    M, ctx = gpu
    A, B = inputs.qd_uniform(24, 40, 0), inputs.qd_uniform(40, 17, 1)
    C = run_qd(M, ctx, A, B, "simple")
    r = error_ratio_exact_python(C, A, B, -208)
    print("qd simple ratio", r)
    assert r <= QD_BOUND


@pytest.mark.parametrize("illcond", [False, True])
def test_qd_block_variants_ragged(gpu, illcond):
    M, ctx = gpu
    m, n, l = 97, 75, 130
    A = inputs.qd_uniform(m, l, 2, illcond=illcond)
    B = inputs.qd_uniform(l, n, 3, illcond=illcond)
    ref = run_qd(M, ctx, A, B, "simple")
    r, _ = error_ratio_full(ref, A, B, -208)
    print("qd illcond" if illcond else "qd uniform", "ratio", r)
    assert r <= QD_BOUND
    for v in M.variants(4):
        C = run_qd(M, ctx, A, B, "block", v)
        for q in range(4):
            assert np.array_equal(C[q], ref[q]), (v, q)


def test_qd_integer_inputs_bit_exact(gpu):
    M, ctx = gpu
    m, n, l = 40, 52, 200
    A = inputs.integers(m, l, 4, 4, bits=60)
    B = inputs.integers(l, n, 4, 5, bits=60)
    Ce = cref.gemm_exact(A, B, out_limbs=4)
    for algo, tile in (("simple", None), ("block", None), ("strassen", {"depth": 1})):
        C = run_qd(M, ctx, A, B, algo, tile)
        for q in range(4):
            assert np.array_equal(C[q], Ce[q]), (algo, q)


def test_qd_strassen_normwise(gpu):
    M, ctx = gpu
    n = 128
    A, B = inputs.qd_uniform(n, n, 6), inputs.qd_uniform(n, n, 7)
    for d in (1, 2):
        C = run_qd(M, ctx, A, B, "strassen", {"depth": d})
        r = normwise_ratio(C, A, B, 4)
        print("qd strassen", d, r, winograd_bound(n, d, QD_UNIT))
        assert r <= winograd_bound(n, d, QD_UNIT)


def test_qd_512_full(gpu):
    """n = 512 (smallest size of the QD workload), every entry."""
    M, ctx = gpu
    n = 512
    A, B = inputs.qd_uniform(n, n, 8), inputs.qd_uniform(n, n, 9)
    C = run_qd(M, ctx, A, B, "block")
    r, _ = error_ratio_full(C, A, B, -208)
    print("qd 512 ratio", r)
    assert r <= QD_BOUND


@pytest.mark.parametrize("algo,tile", [("block", None), ("strassen", {"depth": 1})])
def test_qd_2048_sampled(gpu, algo, tile):
    """n = 2048 (largest size of the QD workload), sampled entries."""
    M, ctx = gpu
    n = 2048
    A, B = inputs.qd_uniform(n, n, 10), inputs.qd_uniform(n, n, 11)
    C = run_qd(M, ctx, A, B, algo, tile)
    pairs = sampled_pairs(n, n, 24)
    errs, mags = sampled_errors(C, A, B, pairs)
    if algo == "block":
        r = max(e / (n * 2.0 ** -208 * g) for e, g in zip(errs, mags))
        assert r <= QD_BOUND
    else:
        r = max(errs) / (np.abs(A[0]).max() * np.abs(B[0]).max() * (1 - 2.0 ** -50))
        assert r <= winograd_bound(n, 1, QD_UNIT)
    print(algo, "sampled ratio", r)
