"""Caller-owned device memory: every device byte a plan, a solve, the lambda
rules and a batched solve use comes from workspaces the caller allocates
(here torch tensors); the library itself allocates none, and too small or
misaligned workspaces are refused with KP_ERR_WORKSPACE."""
import numpy as np
import pytest

import synthetic as S
from oracle import solvers as SV
from tests.gpu_util import rel, require_gpu, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _problem():
    return S.mid_anisotropic(0)


def test_workspace_sizes_grow_with_the_problem():
    require_gpu()
    from paper_2311_15393_amd import kpcg
    small, mid, big = (kpcg.workspace_size(64, 15), kpcg.workspace_size(256, 31),
                       kpcg.workspace_size(1024, 63))
    say(f"workspace bytes: 64/15 {small}, 256/31 {mid}, 1024/63 {big}")
    assert 0 < small < mid < big < 256 * 2 ** 20


def _run_everything(prob, ws_plan, ws_batch, b, x, grid):
    """kp_setup, pcg_solve, gcv_lambda and pcg_solve_batched on caller
    workspaces; returns the solve's x on the host and the batch's infos."""
    import torch
    from paper_2311_15393_amd import KP_FPCG, KP_P16, Plan, solve_batched
    with Plan(prob.psf, prob.n, workspace=ws_plan) as plan:
        _, info = plan.solve(b, prob.lam, tol=1e-7, maxit=500, mode=KP_FPCG | KP_P16, x=x)
        plan.gcv(b, grid)
        xs = [torch.empty_like(b), torch.empty_like(b)]
        _, infos, _ = solve_batched([plan], [b, b], [prob.lam, 2 * prob.lam], [0, 0], tol=1e-6,
                                    maxit=500, mode=KP_FPCG | KP_P16, xs=xs,
                                    workspace=ws_batch)
        torch.cuda.synchronize()
    return info, infos


def test_library_allocates_no_device_memory():
    """After one warm-up pass (code objects, the device's rocBLAS handle and
    the library's streams are created once per process), a second pass of
    setup, solve, GCV and a batched solve on caller workspaces leaves the
    device's free memory exactly unchanged, and gives the same answers."""
    torch = require_gpu()
    from paper_2311_15393_amd import KP_OK, batched_workspace_size, workspace_size
    from paper_2311_15393_amd import Plan
    prob = _problem()
    grid = S.lambda_grid()
    ws_plan = torch.empty(workspace_size(prob.n, prob.k), dtype=torch.uint8, device="cuda")
    b = to_dev(prob.b)
    x = torch.empty_like(b)
    with Plan(prob.psf, prob.n, workspace=ws_plan) as probe:
        nb = batched_workspace_size([probe], [0, 0])
    ws_batch = torch.empty(nb, dtype=torch.uint8, device="cuda")
    info0, _ = _run_everything(prob, ws_plan, ws_batch, b, x, grid)         # warm-up
    first = to_host(x)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    info1, infos = _run_everything(prob, ws_plan, ws_batch, b, x, grid)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    say(f"free device memory before {free0} after {free1} (delta {free1 - free0}); plan "
        f"workspace {ws_plan.numel()} B, batch workspace {nb} B")
    assert free1 == free0
    assert info1.status == KP_OK and all(i.status == KP_OK for i in infos)
    assert np.array_equal(to_host(x), first)
    ref = SV.x_lambda(prob.psf, prob.b.astype(np.float64), prob.lam)
    assert rel(first, ref) <= 1e-4


def test_workspace_refusals():
    """A plan workspace one byte short or misaligned, and a batch workspace
    one byte short, are refused with KP_ERR_WORKSPACE (nothing launched)."""
    torch = require_gpu()
    from paper_2311_15393_amd import (KP_ERR_WORKSPACE, KP_FPCG, KP_P16, KPError, Plan,
                                      batched_workspace_size, solve_batched, workspace_size)
    prob = S.small_gaussian(0)
    need = workspace_size(prob.n, prob.k)
    short = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(KPError) as ei:
        Plan(prob.psf, prob.n, workspace=short)
    assert ei.value.status == KP_ERR_WORKSPACE
    big = torch.empty(need + 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(KPError) as ei:
        Plan(prob.psf, prob.n, workspace=big[8:])
    assert ei.value.status == KP_ERR_WORKSPACE
    b = to_dev(prob.b)
    with Plan(prob.psf, prob.n) as plan:
        nb = batched_workspace_size([plan], [0])
        with pytest.raises(KPError) as ei:
            solve_batched([plan], [b], [prob.lam], [0], mode=KP_FPCG | KP_P16,
                          workspace=torch.empty(nb - 1, dtype=torch.uint8, device="cuda"))
        assert ei.value.status == KP_ERR_WORKSPACE
