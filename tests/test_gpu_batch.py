"""GPU tests of the batched path (many uneven Burgers problems per launch):
batched FWD / block Hessian / GN step against the FP64 oracle, and the batch
invariance property (a problem's result is bitwise the same alone and in a mix)."""
import numpy as np
import pytest

from gpu_util import colwise_relerr, need_gpu, relerr, to_dev, to_np
from oracle import rng as orng
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu

# uneven sizes and windows, ragged observation layouts; the 256-point problem
# uses the banded prior path, the others the spectral one
CFGS = [inputs.burgers_config(256, 50, 4, 10, dt_cfg=1e-3, name='b256'),
        inputs.burgers_config(400, 77, 3, 7, dt_cfg=1e-3, name='b400'),
        inputs.burgers_config(1000, 120, 5, 12, dt_cfg=1e-3, name='b1000'),
        inputs.burgers_config(611, 33, 4, 11, dt_cfg=1e-3, name='b611')]


def _setup(cfgs, seeds=None):
    from oracle.problem import burgers_problem
    from paper_2401_15758_amd import rp4d
    ctx = rp4d.Context(0)
    orcs, probs, trajs = [], [], []
    for i, cfg in enumerate(cfgs):
        orc = burgers_problem(cfg, inputs.draws(cfg, seed=(seeds[i] if seeds else i)))
        p = rp4d.Problem(ctx, cfg)
        p.set_id(100 + i)
        p.set_data(to_dev(orc.xb), to_dev(orc.y.reshape(-1)))
        orcs.append(orc)
        probs.append(p)
        trajs.append(p.traj())
    return ctx, orcs, probs, trajs


def test_batched_fwd_and_hessian_match_oracle():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    J = b.fwd([to_dev(o.xb) for o in orcs], trajs)
    k = 5
    Vs = [np.random.default_rng(10 + i).standard_normal((o.n, k)) for i, o in enumerate(orcs)]
    HVs = b.hessian_block(trajs, [to_dev(v) for v in Vs])
    for i, o in enumerate(orcs):
        otr = o.fwd(o.xb)
        d = o.innovations(otr)
        assert J[i] == pytest.approx(0.5 * np.sum(d * d), rel=1e-12)
        assert relerr(to_np(probs[i].observe(trajs[i])), o.observe(otr)) <= 1e-13
        assert colwise_relerr(to_np(HVs[i]), o.hessian(otr, Vs[i])) <= 1e-12


def test_batched_hessian_matches_single_problem_path():
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    b.fwd([to_dev(o.xb) for o in orcs], trajs, want_J=False)
    Vs = [to_dev(np.random.default_rng(20 + i).standard_normal((o.n, 8))).to(torch.float32) for i, o in enumerate(orcs)]
    HB = b.hessian_block(trajs, Vs)
    for i, p in enumerate(probs):
        HS = p.hessian_block(trajs[i], Vs[i])
        assert colwise_relerr(to_np(HB[i]), to_np(HS)) <= 1e-6   # FP32 sweeps, different prior reduction order


def test_batched_trajectory_serves_single_problem_sweeps_bitwise():
    """A trajectory filled by the batched FWD serves the single-problem path:
    observations and FP64 block Hessians on it are bitwise those on a
    trajectory from rp4d_fwd."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    b.fwd([to_dev(o.xb) for o in orcs], trajs, want_J=False)
    Vs = [to_dev(np.random.default_rng(40 + i).standard_normal((o.n, 5))) for i, o in enumerate(orcs)]
    for i, p in enumerate(probs):
        own = p.traj()
        p.fwd(to_dev(orcs[i].xb), own, want_J=False)
        a = p.hessian_block(trajs[i], Vs[i]).clone()
        c = p.hessian_block(own, Vs[i])
        torch.cuda.synchronize()
        assert torch.equal(p.observe(trajs[i]), p.observe(own)), i
        assert torch.equal(a, c), i


def test_batched_tilings_are_bitwise_identical():
    """Batched sweeps give the same bits with wave regions (the default) and
    with workgroup regions, for the forward sweep and the block Hessian."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    xs = [to_dev(o.xb) for o in orcs]
    Vs = [to_dev(np.random.default_rng(50 + i).standard_normal((o.n, 5))) for i, o in enumerate(orcs)]
    b.fwd(xs, trajs, want_J=False)
    obs0 = [p.observe(t).clone() for p, t in zip(probs, trajs)]
    h0 = [h.clone() for h in b.hessian_block(trajs, Vs)]
    for tiling in [dict(xch=rp4d.XCH_LDS, ppt=2, kc=2, threads=256, steps=16),
                   dict(xch=rp4d.XCH_WAVE, ppt=2, kc=1, threads=64, steps=5),
                   dict(xch=rp4d.XCH_WAVE, ppt=4, kc=2, threads=128, steps=20)]:
        for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
            b.set_tiling(mode, **tiling)
        b.set_tiling(rp4d.MODE_FWD, ppt=tiling["ppt"], threads=tiling["threads"], steps=tiling["steps"],
                     xch=tiling["xch"])
        b.fwd(xs, trajs, want_J=False)
        h = b.hessian_block(trajs, Vs)
        torch.cuda.synchronize()
        for i in range(len(probs)):
            assert torch.equal(probs[i].observe(trajs[i]), obs0[i]), (tiling, i)
            assert torch.equal(h[i], h0[i]), (tiling, i)


def test_batch_invariance_alone_and_in_mix():
    """Each problem's batched block Hessian is bitwise identical whether it runs
    alone or with the other problems."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    b.fwd([to_dev(o.xb) for o in orcs], trajs, want_J=False)
    Vs = [to_dev(np.random.default_rng(30 + i).standard_normal((o.n, 6))) for i, o in enumerate(orcs)]
    mix = [h.clone() for h in b.hessian_block(trajs, Vs)]
    for i, p in enumerate(probs):
        alone = rp4d.Batch(ctx, [p]).hessian_block([trajs[i]], [Vs[i]])[0]
        torch.cuda.synchronize()
        assert torch.equal(alone, mix[i]), i


def _omega_seed(seed, index):
    return (seed ^ ((0x9E3779B97F4A7C15 * (index + 1)) & 0xFFFFFFFFFFFFFFFF)) & 0xFFFFFFFFFFFFFFFF


def test_batched_gn_step_matches_oracle():
    torch = need_gpu()
    from oracle import gn as ogn
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    states = [p.gn_state() for p in probs]
    ell, seed = 12, 77
    infos = b.gn_step(states, sketch=rp4d.NYSTROM, ell=ell, seed=seed, rtol=1e-12)
    for i, (o, p) in enumerate(zip(orcs, probs)):
        # the batch draws Omega on the device from the problem id; the oracle
        # reproduces the same stream with its own generator
        Om = orng.gaussian_matrix(_omega_seed(seed, 100 + i), o.n, ell)
        v1, dv, x1, info = ogn.gn_step(o, np.zeros(o.n), method='nystrom', Omega=Om, rtol=1e-12)
        gv, gx = states[i].get()
        assert infos[i]['J'] == pytest.approx(info['J'], rel=1e-12)
        # at rtol 1e-12 the last iterations are at roundoff: counts may differ by a few
        assert abs(infos[i]['pcg_iters'] - info['pcg']['iters']) <= 3
        assert relerr(to_np(gx), x1) <= 1e-10, i
        c = p.counters()
        assert c['tlm_offline'] == ell and c['tlm_online'] == infos[i]['pcg_iters']


def test_batched_gn_fp32_sketch_and_mix_invariance():
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    states = [p.gn_state() for p in probs]
    Js = []
    for it in range(3):
        infos = b.gn_step(states, sketch=rp4d.NYSTROM, ell=16, seed=5 + it, sketch_dtype=rp4d.F32, rtol=1e-6,
                          reuse_eps=10.0)
        Js.append([inf['J'] for inf in infos])
        assert all(inf['pcg_converged'] for inf in infos)
    for i in range(len(probs)):
        assert Js[1][i] < Js[0][i]
    # the last problem alone, same three steps: bitwise equal final state
    p = probs[-1]
    st = p.gn_state()
    bb = rp4d.Batch(ctx, [p])
    for it in range(3):
        bb.gn_step([st], sketch=rp4d.NYSTROM, ell=16, seed=5 + it, sketch_dtype=rp4d.F32, rtol=1e-6, reuse_eps=10.0)
    _, xa = st.get()
    _, xm = states[-1].get()
    torch.cuda.synchronize()
    # random draws follow the problem id, reductions are per problem: bitwise equal
    assert torch.equal(xa, xm)


# the extremes of batch-64's ranges: n 256 and 4096 (the 4096-point problems at
# the stability-limited step), windows of 50 and 500 steps
EXTREMES = [inputs.burgers_config(256, 50, 4, 10, dt_cfg=1e-3, name='b256-50'),
            inputs.burgers_config(4096, 500, 4, 10, dt_cfg=1e-3, name='b4096-500'),
            inputs.burgers_config(256, 500, 4, 10, dt_cfg=1e-3, name='b256-500'),
            inputs.burgers_config(4096, 50, 4, 10, dt_cfg=1e-3, name='b4096-50')]


def test_batched_gn_step_at_the_extremes_matches_oracle():
    """One batched GN step (32-column Nystrom sketches drawn on the device,
    FP64, rtol 1e-12) over problems at the corners of batch-64's size and window
    ranges, against the oracle per problem: x+ within 1e-10."""
    need_gpu()
    from oracle import gn as ogn
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(EXTREMES, seeds=[11, 12, 13, 14])
    b = rp4d.Batch(ctx, probs)
    states = [p.gn_state() for p in probs]
    ell, seed = 32, 91
    infos = b.gn_step(states, sketch=rp4d.NYSTROM, ell=ell, seed=seed, rtol=1e-12)
    for i, (o, p) in enumerate(zip(orcs, probs)):
        Om = orng.gaussian_matrix(_omega_seed(seed, 100 + i), o.n, ell)
        _, dv, x1, info = ogn.gn_step(o, np.zeros(o.n), method='nystrom', Omega=Om, rtol=1e-12)
        _, gx = states[i].get()
        assert infos[i]['J'] == pytest.approx(info['J'], rel=1e-12), i
        assert infos[i]['pcg_converged'], i
        assert relerr(to_np(gx), x1) <= 1e-10, i


def test_batched_pcg_graph_replay_is_bitwise_eager():
    """With graphs on, the lock-step PCG replays its iteration body captured
    for the current set of unconverged problems (captured again whenever a
    problem drops out; every replay is followed by the eager residual
    read-back).  Uneven problems converge at different iterations, so several
    captures happen; every problem's iteration count and solution must equal
    the all-eager run bit for bit, and stay within 1e-10 of the oracle."""
    torch = need_gpu()
    from oracle import gn as ogn
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    ell, seed = 12, 78
    out = {}
    for graphs in (False, True):
        ctx.set_graphs(graphs)
        states = [p.gn_state() for p in probs]
        infos = b.gn_step(states, sketch=rp4d.NYSTROM, ell=ell, seed=seed, rtol=1e-12)
        torch.cuda.synchronize()
        out[graphs] = ([inf['pcg_iters'] for inf in infos], [s.get()[1].clone() for s in states])
    ctx.set_graphs(False)
    iters = out[False][0]
    assert out[True][0] == iters and min(iters) >= 5 and len(set(iters)) >= 2
    for i in range(len(probs)):
        assert torch.equal(out[True][1][i], out[False][1][i]), i
    for i, o in enumerate(orcs):
        Om = orng.gaussian_matrix(_omega_seed(seed, 100 + i), o.n, ell)
        _, _, x1, _ = ogn.gn_step(o, np.zeros(o.n), method='nystrom', Omega=Om, rtol=1e-12)
        assert relerr(to_np(out[True][1][i]), x1) <= 1e-10, i


def test_single_vector_batched_tiling_entry():
    """The k = 1 tiling entry of a batch (rp4d_batch_set_tiling_k) drives the
    single-vector sweeps and only them: another valid entry gives bitwise the
    same products, an entry too small for its halo fails the k = 1 product but
    not a k = 5 one, and kc > 1 is rejected for it."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx, orcs, probs, trajs = _setup(CFGS)
    b = rp4d.Batch(ctx, probs)
    b.fwd([to_dev(o.xb) for o in orcs], trajs, want_J=False)
    V1 = [to_dev(np.random.default_rng(60 + i).standard_normal((o.n, 1))) for i, o in enumerate(orcs)]
    V5 = [to_dev(np.random.default_rng(70 + i).standard_normal((o.n, 5))) for i, o in enumerate(orcs)]
    ref = [h.clone() for h in b.hessian_block(trajs, V1)]
    for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
        b.set_tiling(mode, k=1, xch=rp4d.XCH_LDS, ppt=1, threads=256, steps=5)
    out = b.hessian_block(trajs, V1)
    torch.cuda.synchronize()
    assert all(torch.equal(x, y) for x, y in zip(out, ref))
    b.set_tiling(rp4d.MODE_ADJ, k=1, xch=rp4d.XCH_WAVE, ppt=1, threads=64, steps=20)
    with pytest.raises(rp4d.Rp4dError):
        b.hessian_block(trajs, V1)
    b.hessian_block(trajs, V5)
    with pytest.raises(rp4d.Rp4dError):
        b.set_tiling(rp4d.MODE_TLM, k=1, kc=2)
    for mode in (rp4d.MODE_TLM, rp4d.MODE_ADJ):
        b.set_tiling(mode, k=1)
    torch.cuda.synchronize()
