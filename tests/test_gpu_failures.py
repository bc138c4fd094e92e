"""Error paths forced from the host: a failed workspace allocation
(MPG_ERR_NOMEM) and a failed kernel launch (MPG_ERR_HIP) are reported with
their detail, leave the context usable, and a tuner trial whose workspace
cannot be allocated is skipped (the tuner falls back to the candidates that
need none).  Nothing here reaches the GPU in a failing state: the injected
failures return before any HIP call is made."""
import numpy as np
import pytest
import torch

from paper_1710_01839_amd import inputs

pytestmark = pytest.mark.gpu


def _operands(M, n=96, seed=70):
    A, B = inputs.dd_uniform(n, n, seed), inputs.dd_uniform(n, n, seed + 1)
    return A, B, M.to_device(A), M.to_device(B), M.empty_like_limbs(n, n, 2)


def test_workspace_allocation_failure(gpu):
    """Strassen needs workspace: with allocations failing the call returns
    MPG_ERR_NOMEM with the size in the message; afterwards it runs and agrees
    bitwise with a fresh run."""
    M, ctx = gpu
    fresh = M.Context(0)      # a context with no workspace yet
    try:
        A, B, Ad, Bd, C = _operands(M)
        fresh.inject("alloc", 1)
        with pytest.raises(M.MpgemmError) as ei:
            M.mpgemm_dd(fresh, Ad, Bd, C, algo="strassen", tile={"depth": 1})
        assert ei.value.status == M.MPG_ERR_NOMEM
        assert "workspace allocation" in str(ei.value)
        # the block kernel needs no workspace: unaffected by a pending injection
        fresh.inject("alloc", 1)
        M.mpgemm_dd(fresh, Ad, Bd, C, algo="block")
        fresh.inject("alloc", 0)
        M.mpgemm_dd(fresh, Ad, Bd, C, algo="strassen", tile={"depth": 1})
        torch.cuda.synchronize()
        got = M.to_host(C)
        C2 = M.empty_like_limbs(96, 96, 2)
        M.mpgemm_dd(ctx, Ad, Bd, C2, algo="strassen", tile={"depth": 1})
        torch.cuda.synchronize()
        want = M.to_host(C2)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
        # the split product's workspace too
        fresh2 = M.Context(0)
        try:
            fresh2.inject("alloc", 1)
            with pytest.raises(M.MpgemmError) as ei:
                M.mpgemm_dd_ozaki(fresh2, Ad, Bd, C, 0, "crt")
            assert ei.value.status == M.MPG_ERR_NOMEM
        finally:
            fresh2.close()
    finally:
        fresh.close()


def test_launch_failure_reported(gpu):
    """A failed launch returns MPG_ERR_HIP naming the HIP error and the step;
    the next call runs normally."""
    M, ctx = gpu
    A, B, Ad, Bd, C = _operands(M, seed=72)
    ctx.inject("launch", 1)
    with pytest.raises(M.MpgemmError) as ei:
        M.mpgemm_dd(ctx, Ad, Bd, C, algo="block")
    assert ei.value.status == M.MPG_ERR_HIP
    assert "hipErrorLaunchFailure" in str(ei.value) and "block kernel" in str(ei.value)
    # a multi-launch path fails at its first launch and returns
    ctx.inject("launch", 1)
    with pytest.raises(M.MpgemmError) as ei:
        M.mpgemm_dd(ctx, Ad, Bd, C, algo="strassen", tile={"depth": 1})
    assert ei.value.status == M.MPG_ERR_HIP and "Strassen operands" in str(ei.value)
    M.mpgemm_dd(ctx, Ad, Bd, C, algo="block")
    torch.cuda.synchronize()
    C2 = M.empty_like_limbs(96, 96, 2)
    M.mpgemm_dd(ctx, Ad, Bd, C2, algo="simple")
    torch.cuda.synchronize()
    got, want = M.to_host(C), M.to_host(C2)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_tuner_skips_candidates_without_workspace(gpu):
    """With every workspace allocation failing, the exhaustive tuner skips
    Strassen and the split products and picks among simple and block."""
    M, ctx = gpu
    fresh = M.Context(0)
    try:
        T = M.Tuner(fresh)
        n = 256
        cands = M.candidates("dd", n, n, n)
        fresh.inject("alloc", 10 ** 6)
        r = T.tune("dd", n, n, n, "exhaustive")
        fresh.inject("alloc", 0)
        no_ws = [a for a, _ in cands if a in (M.MPG_SIMPLE, M.MPG_BLOCK)]
        assert r["trials"] == len(no_ws) < len(cands)
        assert r["algo"] in (M.MPG_SIMPLE, M.MPG_BLOCK)
        r2 = T.tune("dd", n, n, n, "exhaustive")
        assert r2["trials"] == len(cands)
    finally:
        fresh.close()
