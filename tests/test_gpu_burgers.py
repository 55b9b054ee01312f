"""GPU parity of the Burgers block operators (HIP library through the C ABI) with
the FP64 CPU oracle: prior square root, FWD trajectory and cost, TLM (A V), ADJ
(A^T W), the block Hessian (I + A^T A) V, the gradient; plus determinism across
sweep tilings and checkpointing, the FP32 sweep error, and edge cases."""
import numpy as np
import pytest

from gpu_util import Pair, colwise_relerr, need_gpu, relerr, to_dev, to_np
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu

# FP64 parity tolerance for the operators: the GPU and the oracle differ only in
# rounding order; over <= 500 RK4 steps the relative difference stays ~1e-14.
TOL_OP = 1e-12

RAGGED = inputs.burgers_config(200, 37, 3, 7, dt_cfg=1e-3, name='burgers-200-ragged')
TINY = inputs.burgers_config(16, 5, 5, 2, dt_cfg=1e-3, L_b=0.2, name='burgers-16')


@pytest.fixture(scope="module")
def small():
    need_gpu()
    return Pair(inputs.CFG_SMALL)


@pytest.fixture(scope="module")
def ragged():
    need_gpu()
    return Pair(RAGGED, seed=3)


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("n,k", [(128, 3), (200, 1), (4096, 5)])
def test_bhalf_parity(n, k):
    torch = need_gpu()
    from oracle import prior
    from paper_2401_15758_amd import rp4d
    cfg = inputs.burgers_config(n, 10, 4, 5, dt_cfg=1e-7 if n > 1000 else 1e-4)
    ctx = rp4d.Context(0)
    p = rp4d.Problem(ctx, cfg)
    V = _rand((n, k), 11)
    U = to_np(p.bhalf(to_dev(V)))
    ref = prior.bhalf_1d(V, 1.0 / n, cfg['sigma_b'], cfg['L_b'])
    assert relerr(U, ref) <= 1e-13
    U32 = to_np(p.bhalf(to_dev(V, torch.float32)))
    assert relerr(U32, ref) <= 1e-6


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_fwd_observations_and_cost(which, request):
    pr = request.getfixturevalue(which)
    obs = to_np(pr.gpu.observe(pr.traj))
    ref = pr.orc.observe(pr.otraj)
    assert relerr(obs, ref) <= 1e-13
    d = pr.orc.innovations(pr.otraj)
    assert pr.Jobs == pytest.approx(0.5 * float(np.sum(d * d)), rel=1e-12)


@pytest.mark.parametrize("which,k", [("small", 20), ("small", 1), ("ragged", 7)])
def test_tlm_parity(which, k, request):
    pr = request.getfixturevalue(which)
    V = _rand((pr.orc.n, k), 21)
    Z = to_np(pr.gpu.tlm(pr.traj, to_dev(V)))
    ref = pr.orc.A(pr.otraj, V).reshape(Z.shape)
    assert colwise_relerr(Z.reshape(-1, k), ref.reshape(-1, k)) <= TOL_OP


@pytest.mark.parametrize("which,k", [("small", 20), ("ragged", 5)])
def test_adj_parity(which, k, request):
    pr = request.getfixturevalue(which)
    W = _rand((pr.orc.n_t, pr.orc.n_obs, k), 31)
    U = to_np(pr.gpu.adj(pr.traj, to_dev(W)))
    ref = pr.orc.AT(pr.otraj, W)
    assert colwise_relerr(U, ref) <= TOL_OP


@pytest.mark.parametrize("which,k,ident", [("small", 20, True), ("small", 3, False), ("ragged", 9, True)])
def test_hessian_block_parity(which, k, ident, request):
    pr = request.getfixturevalue(which)
    V = _rand((pr.orc.n, k), 41)
    HV = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V), add_identity=ident))
    ref = pr.orc.hessian(pr.otraj, V) if ident else pr.orc.misfit_hessian(pr.otraj, V)
    assert colwise_relerr(HV, ref) <= TOL_OP


def test_dot_product_test_on_gpu(small):
    pr = small
    V = _rand((pr.orc.n, 4), 51)
    W = _rand((pr.orc.n_t, pr.orc.n_obs, 4), 52)
    AV = to_np(pr.gpu.tlm(pr.traj, to_dev(V)))
    ATW = to_np(pr.gpu.adj(pr.traj, to_dev(W)))
    lhs, rhs = np.sum(AV * W), np.sum(V * ATW)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(AV) * np.linalg.norm(W)


def test_gradient_parity(small):
    pr = small
    v = 0.1 * _rand(pr.orc.n, 61)
    # trajectory at x = x_b + Gamma^{1/2} v on both sides
    x = to_np(pr.gpu.bhalf(to_dev(v.reshape(-1, 1)))).reshape(-1) + pr.orc.xb
    tr = pr.gpu.traj()
    pr.gpu.fwd(to_dev(x), tr)
    g = to_np(pr.gpu.gradient(tr, to_dev(v)))
    _, gref, _, _ = pr.orc.cost_grad(v)
    assert relerr(g, gref) <= 1e-12


def test_fp32_sweeps_error_is_stated(small):
    torch = need_gpu()
    pr = small
    V = _rand((pr.orc.n, 20), 71)
    H32 = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V, torch.float32), add_identity=False))
    ref = pr.orc.misfit_hessian(pr.otraj, V)
    # FP32 sweeps: relative error of H V against the FP64 oracle (single precision over 50 steps)
    assert colwise_relerr(H32, ref) <= 1e-4


def test_tilings_are_bitwise_identical(ragged):
    torch = need_gpu()
    pr = ragged
    V = to_dev(_rand((pr.orc.n, 9), 81))
    base = pr.gpu.hessian_block(pr.traj, V).clone()
    from paper_2401_15758_amd import rp4d
    L, Wv = rp4d.XCH_LDS, rp4d.XCH_WAVE
    # workgroup regions, then wave regions (64 * ppt points each; the last one
    # wraps the 200-point ring more than twice)
    for ppt, kc, threads, tile, steps, xch in [(1, 1, 128, 50, 1, L), (2, 2, 128, 64, 5, L), (4, 4, 128, 200, 7, L),
                                               (2, 4, 256, 17, 3, L), (4, 1, 64, 100, 2, L),
                                               (1, 1, 64, 16, 5, Wv), (2, 2, 128, 40, 9, Wv),
                                               (4, 1, 256, 100, 15, Wv), (2, 4, 256, 30, 3, Wv),
                                               (1, 4, 128, 7, 6, Wv), (8, 1, 64, 150, 25, Wv)]:
        pr.gpu.set_sweep_tiling(k=9, ppt=ppt, kc=kc, threads=threads, tile=tile, steps=steps, xch=xch)
        assert pr.gpu.get_sweep_tiling(k=9)["xch"] == xch
        out = pr.gpu.hessian_block(pr.traj, V)
        torch.cuda.synchronize()
        assert torch.equal(out, base), (ppt, kc, threads, tile, steps, xch)
    pr.gpu.set_sweep_tiling(k=9)


def test_wave_tiling_rejects_short_regions(ragged):
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = ragged
    V = to_dev(_rand((pr.orc.n, 2), 82))
    # 64 * 1 points cannot hold a 20-point tile plus two 24-point halos
    pr.gpu.set_sweep_tiling(k=2, ppt=1, kc=1, threads=64, tile=20, steps=5, xch=rp4d.XCH_WAVE)
    with pytest.raises(rp4d.Rp4dError):
        pr.gpu.hessian_block(pr.traj, V)
    # wave workgroups group at most 4 waves
    pr.gpu.set_sweep_tiling(k=2, ppt=1, kc=1, threads=512, tile=16, steps=5, xch=rp4d.XCH_WAVE)
    with pytest.raises(rp4d.Rp4dError):
        pr.gpu.hessian_block(pr.traj, V)
    pr.gpu.set_sweep_tiling(k=2)
    torch.cuda.synchronize()


def test_fwd_tilings_are_bitwise_identical(ragged):
    """The forward sweep's tiling (autotuned like the block sweeps) changes no bit
    of the trajectory: observations and the Hessian built on it are identical."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = ragged
    V = to_dev(_rand((pr.orc.n, 3), 83))
    obs0 = pr.gpu.observe(pr.traj).clone()
    hv0 = pr.gpu.hessian_block(pr.traj, V).clone()
    tr = pr.gpu.traj()
    L, Wv = rp4d.XCH_LDS, rp4d.XCH_WAVE
    for ppt, threads, tile, steps, xch in [(1, 128, 50, 4, L), (2, 192, 100, 8, L), (8, 64, 200, 12, L),
                                           (4, 256, 200, 25, L), (1, 64, 24, 4, Wv), (2, 128, 56, 8, Wv),
                                           (4, 256, 120, 16, Wv), (8, 64, 200, 30, Wv)]:
        pr.gpu.set_sweep_tiling(mode=rp4d.MODE_FWD, ppt=ppt, threads=threads, tile=tile, steps=steps, xch=xch)
        got = pr.gpu.get_sweep_tiling(mode=rp4d.MODE_FWD)
        assert got["steps"] == steps and got["xch"] == xch
        pr.gpu.fwd(pr.xb_dev, tr, want_J=False)
        torch.cuda.synchronize()
        assert torch.equal(pr.gpu.observe(tr), obs0), (ppt, threads, tile, steps, xch)
        assert torch.equal(pr.gpu.hessian_block(tr, V), hv0), (ppt, threads, tile, steps, xch)
    pr.gpu.set_sweep_tiling(mode=rp4d.MODE_FWD)


def test_checkpointed_trajectory_bitwise(small):
    torch = need_gpu()
    pr = small
    ck = Pair(inputs.CFG_SMALL, ckpt_every=7, ctx=pr.ctx)
    V = to_dev(_rand((pr.orc.n, 6), 91))
    a = pr.gpu.hessian_block(pr.traj, V)
    b = ck.gpu.hessian_block(ck.traj, V)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(pr.gpu.observe(pr.traj), ck.gpu.observe(ck.traj))


def test_tiny_problem_and_single_vector():
    need_gpu()
    pr = Pair(TINY, seed=5)
    V = _rand((16, 1), 101)
    HV = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V)))
    assert colwise_relerr(HV, pr.orc.hessian(pr.otraj, V)) <= TOL_OP


def test_unstable_step_rejected():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    cfg = dict(inputs.CFG_LARGE)
    cfg['dt'] = cfg['dt_cfg']        # the literal configured step: 4 nu dt/dx^2 = 16.8
    with pytest.raises(rp4d.Rp4dError) as e:
        rp4d.Problem(rp4d.Context(0), cfg)
    assert e.value.code == rp4d.EUNSTABLE


def test_bad_shapes_rejected(small):
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    with pytest.raises(ValueError):
        small.gpu.hessian_block(small.traj, torch.zeros(7, 2, dtype=torch.float64, device="cuda"))
    with pytest.raises(rp4d.Rp4dError):
        small.gpu.set_sweep_tiling(k=2, ppt=3, kc=1, threads=64, tile=16, steps=1)
        small.gpu.hessian_block(small.traj, torch.zeros(128, 2, dtype=torch.float64, device="cuda"))
    small.gpu.set_sweep_tiling(k=2)


def test_large_config_sampled_columns():
    """burgers-4096 (n=4096, 500 steps, k=64) in the launch configuration the
    benchmark times; the oracle checks 3 sampled columns."""
    need_gpu()
    from paper_2401_15758_amd import autotune
    pr = Pair(inputs.CFG_LARGE)
    for k in (64, 1):
        autotune.apply_cached(pr.gpu, inputs.CFG_LARGE["nsteps"], k)
    V = inputs.omega(4096, 64, seed=1000)
    HV = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V)))
    cols = [0, 31, 63]
    ref = pr.orc.hessian(pr.otraj, V[:, cols])
    assert colwise_relerr(HV[:, cols], ref) <= 1e-11
    obs = to_np(pr.gpu.observe(pr.traj))
    assert relerr(obs, pr.orc.observe(pr.otraj)) <= 1e-12


@pytest.mark.parametrize("cfg", [inputs.CFG_SMALL, RAGGED])
def test_synthesis_parity(cfg):
    """Device synthesis x_b = x_true + Gamma^{1/2} xi, y = O M(x_true) + sigma_o eta
    against the oracle's synthesis from the same draws."""
    need_gpu()
    from oracle.problem import burgers_problem
    from paper_2401_15758_amd import rp4d
    d = inputs.draws(cfg, seed=4)
    orc = burgers_problem(cfg, d)
    p = rp4d.Problem(rp4d.Context(0), cfg)
    xb, y = p.synthesize(to_dev(d['x_true']), to_dev(d['xi']), to_dev(d['eta'].reshape(-1)))
    assert relerr(to_np(xb), orc.xb) <= 1e-14
    assert relerr(to_np(y), orc.y) <= 1e-13


def test_span_timing_counts_like_per_launch_timing(small):
    """Timing mode 2 (one event pair per sweep) reports the same launches and
    flops as per-launch timing, and a duration of the same order."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = small
    V = to_dev(_rand((pr.orc.n, 4), 112))
    stats = {}
    for mode in (rp4d.TIMING_LAUNCH, rp4d.TIMING_SPAN):
        pr.ctx.set_timing(mode)
        pr.gpu.hessian_block(pr.traj, V)
        stats[mode] = [pr.ctx.kernel_stats(k) for k in (rp4d.K_TLM, rp4d.K_ADJ)]
        pr.ctx.set_timing(False)
    for a, b in zip(stats[rp4d.TIMING_LAUNCH], stats[rp4d.TIMING_SPAN]):
        assert a['launches'] == b['launches'] and a['alg_flops'] == b['alg_flops']
        assert b['total_ms'] > 0 and 0.2 * a['total_ms'] < b['total_ms'] < 5 * a['total_ms']


def test_kernel_timing_counts_launches(small):
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = small
    pr.ctx.set_timing(True)
    V = to_dev(_rand((pr.orc.n, 4), 111))
    pr.gpu.hessian_block(pr.traj, V)
    st = pr.ctx.kernel_stats(rp4d.K_TLM)
    sa = pr.ctx.kernel_stats(rp4d.K_ADJ)
    pr.ctx.set_timing(False)
    t = pr.gpu.get_sweep_tiling(rp4d.F64, 4)
    launches = -(-50 // t['steps'])
    assert st['launches'] == launches and sa['launches'] == launches
    assert st['total_ms'] > 0 and st['alg_flops'] == pytest.approx(50 * 128 * (36 * 4 + 48))


@pytest.mark.parametrize("k", [301, 4096])
def test_wide_blocks_match_column_slices(small, k):
    """Blocks of 301 columns (not a multiple of any vector group) and of the
    largest accepted 4096 columns: every column equals the oracle's product
    on sampled columns, and the block equals its own column slices computed as
    separate smaller blocks (the column grouping does not touch any value)."""
    torch = need_gpu()
    pr = small
    V = _rand((pr.orc.n, k), 7 + k)
    HV = pr.gpu.hessian_block(pr.traj, to_dev(V))
    cols = np.random.default_rng(k).choice(k, size=6, replace=False)
    ref = pr.orc.hessian(pr.otraj, V[:, cols])
    assert colwise_relerr(to_np(HV)[:, cols], ref) <= TOL_OP
    lo, hi = 64, min(k, 64 + 37)
    part = pr.gpu.hessian_block(pr.traj, to_dev(np.ascontiguousarray(V[:, lo:hi])))
    assert colwise_relerr(to_np(HV)[:, lo:hi], to_np(part)) <= 1e-14


def test_block_wider_than_4096_rejected(small):
    need_gpu()
    from paper_2401_15758_amd import rp4d
    with pytest.raises(rp4d.Rp4dError):
        small.gpu.hessian_block(small.traj, to_dev(np.zeros((small.orc.n, 4097))))
