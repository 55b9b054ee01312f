"""The context's HBM budget (rp4d_ctx_create's hbm_budget_bytes): device bytes
held through a context's objects are counted as they are allocated and freed,
an allocation beyond the budget fails with ENOMEM and leaves every object
usable, and freeing makes room again."""
import numpy as np
import pytest

from gpu_util import need_gpu, to_dev
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu

MIB = 1 << 20


def test_usage_is_counted_and_returned():
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx = rp4d.Context(0)
    assert ctx.hbm() == {"used": 0, "budget": 0}
    cfg = inputs.CFG_LARGE
    p = rp4d.Problem(ctx, cfg)
    after_problem = ctx.hbm()["used"]
    assert after_problem > 0
    tr = p.traj()
    traj_bytes = ctx.hbm()["used"] - after_problem
    assert traj_bytes >= 8 * cfg["n"] * (cfg["nsteps"] + 1)           # every state stored
    d = inputs.draws(cfg, seed=0)
    xb, y = p.synthesize(to_dev(d["x_true"]), to_dev(d["xi"]), to_dev(d["eta"].reshape(-1)))
    p.set_data(xb, y.reshape(-1))
    p.fwd(xb, tr)
    V = to_dev(np.random.default_rng(1).standard_normal((cfg["n"], 16)))
    p.hessian_block(tr, V)                                              # sweep workspaces grow
    torch.cuda.synchronize()
    assert ctx.hbm()["used"] > after_problem + traj_bytes
    tr.close()
    p.close()
    assert ctx.hbm()["used"] == 0


def test_budget_rejects_and_recovers():
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    cfg = inputs.CFG_LARGE
    traj_bytes = 8 * cfg["n"] * (cfg["nsteps"] + 1)
    ctx = rp4d.Context(0, hbm_budget=64 * MIB)
    assert ctx.hbm()["budget"] == 64 * MIB
    p = rp4d.Problem(ctx, cfg)
    trajs = []
    with pytest.raises(rp4d.Rp4dError) as e:
        for _ in range(8):
            trajs.append(p.traj())
    assert e.value.code == rp4d.ENOMEM and "budget" in str(e.value)
    assert 2 <= len(trajs) < 8
    used = ctx.hbm()["used"]
    assert used <= 64 * MIB and used + traj_bytes > 64 * MIB
    # the objects still work, and freeing one trajectory makes room for another
    d = inputs.draws(cfg, seed=0)
    xb, y = p.synthesize(to_dev(d["x_true"]), to_dev(d["xi"]), to_dev(d["eta"].reshape(-1)))
    p.set_data(xb, y.reshape(-1))
    J = p.fwd(xb, trajs[0])
    assert np.isfinite(J)
    used = ctx.hbm()["used"]
    trajs.pop().close()
    assert ctx.hbm()["used"] < used
    trajs.append(p.traj())
    assert ctx.hbm()["used"] == used
    for t in trajs:
        t.close()
    p.close()
    torch.cuda.synchronize()
    assert ctx.hbm()["used"] == 0
