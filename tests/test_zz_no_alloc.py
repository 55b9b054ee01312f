"""The no-allocation block Hessian (rp4d_hessian_block_noalloc, workspaces in a
static per-GPU scratch array) against rp4d_hessian_block: bitwise equal
results on consecutive calls that shrink (a large block, then a smaller one on
another problem, then FP32 sweeps on a checkpointed trajectory), no device
memory taken by the call, and the size and model limits reported as errors."""
import numpy as np
import pytest

from gpu_util import Pair, need_gpu, to_dev
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu


def _block(n, k, seed, dtype=None):
    import torch
    V = to_dev(np.random.default_rng(seed).standard_normal((n, k)))
    return V.to(dtype) if dtype is not None else V


def test_noalloc_matches_hessian_block_on_shrinking_calls():
    torch = need_gpu()
    from paper_2401_15758_amd import autotune, rp4d
    ctx = rp4d.Context(0)
    big = Pair(inputs.CFG_LARGE, ctx=ctx)
    for k in (64, 1):
        autotune.apply_cached(big.gpu, inputs.CFG_LARGE["nsteps"], k)
    small = Pair(inputs.CFG_SMALL, ctx=ctx)
    ck = Pair(inputs.burgers_config(600, 90, 5, 9, dt_cfg=1e-3, name="b600"), ctx=ctx, ckpt_every=7)
    cases = [(big, 64, None), (small, 5, None), (ck, 3, torch.float32), (big, 2, None)]
    for i, (pr, k, dt) in enumerate(cases):
        V = _block(pr.orc.n, k, 100 + i, dt)
        got = pr.gpu.hessian_block_noalloc(pr.traj, V)
        ref = pr.gpu.hessian_block(pr.traj, V)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (i, k)
        assert torch.isfinite(got).all()


def test_noalloc_takes_no_device_memory():
    """On a problem that has never run a block product, rp4d_hessian_block
    grows its workspaces (visible in the device's free memory); the
    no-allocation call leaves the free memory as it was."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx = rp4d.Context(0)
    warm = Pair(inputs.CFG_LARGE, ctx=ctx)
    V = _block(warm.orc.n, 64, 7)
    HV = torch.empty_like(V)
    warm.gpu.hessian_block_noalloc(warm.traj, V, HV)        # code objects loaded, scratch resolved
    torch.cuda.synchronize()
    fresh = Pair(inputs.CFG_LARGE, ctx=ctx)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    fresh.gpu.hessian_block_noalloc(fresh.traj, V, HV)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    ref = fresh.gpu.hessian_block(fresh.traj, V)
    torch.cuda.synchronize()
    assert torch.equal(HV, ref)


def test_noalloc_limits_are_errors():
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx = rp4d.Context(0)
    pr = Pair(inputs.CFG_LARGE, ctx=ctx)
    V = torch.zeros((pr.orc.n, 1024), dtype=torch.float64, device="cuda")
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.hessian_block_noalloc(pr.traj, V)             # 1024 columns: about 200 MiB of workspace
    assert e.value.code == rp4d.EINVAL and "64 MiB" in str(e.value)
    b = Pair(inputs.bve_config(32, nsteps=4, obs_stride=8, obs_every=2, L_cells=3.0, ell=4), ctx=ctx)
    with pytest.raises(rp4d.Rp4dError) as e:
        b.gpu.hessian_block_noalloc(b.traj, torch.zeros((b.orc.n, 2), dtype=torch.float64, device="cuda"))
    assert e.value.code == rp4d.EINVAL
    # the problem is still usable afterwards, through both entry points
    W = _block(pr.orc.n, 4, 9)
    assert torch.equal(pr.gpu.hessian_block_noalloc(pr.traj, W), pr.gpu.hessian_block(pr.traj, W))
