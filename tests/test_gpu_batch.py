"""Batched uneven DD products in one persistent launch and in a replayed HIP
graph: bitwise equal to the single-problem kernels (same tile routine),
within the DD bound of the oracle, valid across replays and updates."""
import numpy as np
import pytest
import torch

from paper_1710_01839_amd import inputs
from tests.helpers import error_ratio_full

pytestmark = pytest.mark.gpu


def make_batch(M, shapes, seed):
    probs, host = [], []
    for i, (m, n, l) in enumerate(shapes):
        A = inputs.dd_uniform(m, l, seed + 3 * i)
        B = inputs.dd_uniform(l, n, seed + 3 * i + 1)
        Ad, Bd = M.to_device(A), M.to_device(B)
        C = tuple(torch.full((m, n), np.nan, dtype=torch.float64, device="cuda") for _ in range(2))
        probs.append((Ad, Bd, C))
        host.append((A, B))
    return probs, host


def reference(M, ctx, probs, tile):
    out = []
    for A, B, _ in probs:
        C = M.empty_like_limbs(A[0].shape[0], B[0].shape[1], 2)
        M.mpgemm_dd(ctx, A, B, C, algo="block", tile=tile)
        out.append(C)
    torch.cuda.synchronize()
    return [M.to_host(C) for C in out]


def same(got, want):
    return all(np.array_equal(g[0], w[0]) and np.array_equal(g[1], w[1]) for g, w in zip(got, want))


SHAPES = [(1, 1, 1), (3, 70, 5), (64, 64, 64), (100, 37, 250), (17, 130, 9), (65, 1, 33),
          (200, 150, 120), (31, 33, 1), (8, 8, 300), (129, 95, 64)]


@pytest.mark.parametrize("variant", [None, 0, 1, 6, 7])
def test_persistent_matches_single_kernels(gpu, variant):
    M, ctx = gpu
    tile = None if variant is None else M.variants(2)[variant]
    probs, host = make_batch(M, SHAPES, 100)
    M.mpgemm_dd_batched(ctx, probs, tile)
    torch.cuda.synchronize()
    got = [M.to_host(C) for _, _, C in probs]
    want = reference(M, ctx, probs, tile if tile is not None else M.variants(2)[1])
    assert same(got, want)
    for (A, B), C in zip(host[:4], got[:4]):
        r, _ = error_ratio_full(C, A, B, -104)
        assert r <= 8.0


def test_back_to_back_calls(gpu):
    """Several batched calls queued without host synchronisation (descriptor
    slots alternate; the third call reuses the first call's slot): every
    batch equals the single-problem kernels bit for bit."""
    M, ctx = gpu
    batches = [make_batch(M, SHAPES[k:] + SHAPES[:k], 200 + 50 * k)[0] for k in range(4)]
    for probs in batches:
        M.mpgemm_dd_batched(ctx, probs, None)
    torch.cuda.synchronize()
    for probs in batches:
        got = [M.to_host(C) for _, _, C in probs]
        assert same(got, reference(M, ctx, probs, M.variants(2)[1]))


def test_graph_replays_and_updates(gpu):
    M, ctx = gpu
    probs, host = make_batch(M, SHAPES, 200)
    plan = M.BatchPlan(ctx, probs)
    want = reference(M, ctx, probs, M.variants(2)[1])
    for rep in range(3):
        for _, _, C in probs:          # eager work between replays
            C[0].fill_(np.nan)
            C[1].fill_(np.nan)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert same([M.to_host(C) for _, _, C in probs], want), rep
    # new shapes and pointers, same count: the captured graph stays valid
    shapes2 = [(n, l, m) for (m, n, l) in SHAPES]
    probs2, _ = make_batch(M, shapes2, 300)
    plan.update(probs2)
    want2 = reference(M, ctx, probs2, M.variants(2)[1])
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        assert same([M.to_host(C) for _, _, C in probs2], want2), rep
    plan.close()


def test_zero_l_and_empty_problems(gpu):
    M, ctx = gpu
    A = tuple(torch.empty((4, 0), dtype=torch.float64, device="cuda") for _ in range(2))
    B = tuple(torch.empty((0, 5), dtype=torch.float64, device="cuda") for _ in range(2))
    C = tuple(torch.full((4, 5), 9.0, dtype=torch.float64, device="cuda") for _ in range(2))
    probs, _ = make_batch(M, [(10, 12, 7)], 400)
    M.mpgemm_dd_batched(ctx, probs + [(A, B, C)])
    torch.cuda.synchronize()
    assert float(C[0].abs().max()) == 0.0 and float(C[1].abs().max()) == 0.0


def test_config_512_uneven(gpu):
    """512 problems, m, n, l log-uniform in [16, 512], one graph replay."""
    M, ctx = gpu
    shapes = inputs.batch_shapes(512)
    probs, host = make_batch(M, shapes, 1000)
    plan = M.BatchPlan(ctx, probs)
    plan.launch()
    torch.cuda.synchronize()
    got = [M.to_host(C) for _, _, C in probs]
    want = reference(M, ctx, probs, M.variants(2)[1])
    assert same(got, want)
    for k in (0, 100, 511):
        r, _ = error_ratio_full(got[k], host[k][0], host[k][1], -104)
        assert r <= 8.0
    plan.close()
