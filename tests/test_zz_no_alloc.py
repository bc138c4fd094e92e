"""The allocation-free batched product: the same results as
mpgemm_dd_batched (bitwise: the same persistent kernel and tile routine) on
two calls in a row, the second with fewer and smaller problems, with every
workspace allocation of its context made to fail; the problem-count limit is
an argument error."""
import numpy as np
import pytest
import torch

from paper_1710_01839_amd import inputs
from tests.helpers import error_ratio_full

pytestmark = pytest.mark.gpu


def _batch(M, shapes, seed):
    probs, host = [], []
    for i, (m, n, l) in enumerate(shapes):
        A = inputs.dd_uniform(m, l, seed + 3 * i)
        B = inputs.dd_uniform(l, n, seed + 3 * i + 1)
        C = tuple(torch.full((m, n), np.nan, dtype=torch.float64, device="cuda") for _ in range(2))
        probs.append((M.to_device(A), M.to_device(B), C))
        host.append((A, B))
    return probs, host


def _copy_outputs(M, probs):
    out = []
    for A, B, _ in probs:
        C = tuple(torch.full((A[0].shape[0], B[0].shape[1]), np.nan, dtype=torch.float64, device="cuda")
                  for _ in range(2))
        out.append((A, B, C))
    return out


def _same(M, p, q):
    for (_, _, C1), (_, _, C2) in zip(p, q):
        a, b = M.to_host(C1), M.to_host(C2)
        if not (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])):
            return False
    return True


FIRST = [(1, 1, 1), (3, 70, 5), (64, 64, 64), (100, 37, 250), (17, 130, 9), (65, 1, 33),
         (200, 150, 120), (31, 33, 1), (8, 8, 300), (129, 95, 64), (257, 190, 77), (40, 300, 200)]
SECOND = [(5, 9, 3), (33, 17, 40), (2, 64, 1), (70, 20, 15)]


@pytest.mark.parametrize("variant", [None, 7])
def test_noalloc_matches_batched_twice(gpu, variant):
    M, ctx = gpu
    tile = None if variant is None else M.variants(2)[variant]
    fresh = M.Context(0)
    try:
        fresh.inject("alloc", 10 ** 6)   # any workspace allocation would fail the call
        p1, h1 = _batch(M, FIRST, 300)
        p2, h2 = _batch(M, SECOND, 400)
        # two calls in a row on one stream, no host synchronisation between
        M.mpgemm_dd_batched_noalloc(fresh, p1, tile)
        M.mpgemm_dd_batched_noalloc(fresh, p2, tile)
        torch.cuda.synchronize()
        r1, r2 = _copy_outputs(M, p1), _copy_outputs(M, p2)
        M.mpgemm_dd_batched(ctx, r1, tile)
        M.mpgemm_dd_batched(ctx, r2, tile)
        torch.cuda.synchronize()
        assert _same(M, p1, r1) and _same(M, p2, r2)
        for (A, B), (_, _, C) in list(zip(h1, p1))[:5] + list(zip(h2, p2)):
            r, _ = error_ratio_full(M.to_host(C), A, B, -104)
            assert r <= 8.0
        fresh.inject("alloc", 0)
    finally:
        fresh.close()


def test_noalloc_limits(gpu):
    M, ctx = gpu
    M.mpgemm_dd_batched_noalloc(ctx, [])           # empty batch: no-op
    A = M.to_device(inputs.dd_uniform(2, 2, 1))
    C = M.empty_like_limbs(2, 2, 2)
    with pytest.raises(M.MpgemmError) as ei:
        M.mpgemm_dd_batched_noalloc(ctx, [(A, A, C)] * 8193)
    assert ei.value.status == M.MPG_ERR_ARG
    # an argument error in one problem (C overlapping A) is reported before
    # anything runs
    with pytest.raises(M.MpgemmError) as ei:
        M.mpgemm_dd_batched_noalloc(ctx, [(A, A, C), (A, A, A)])
    assert ei.value.status == M.MPG_ERR_ALIAS
