"""GPU parity of the barotropic-vorticity path (2-D model) with the FP64 oracle:
the spectral inverse Laplacian and the separable prior square root, the RK4
trajectory and cost, the TLM / ADJ block sweeps (both row-stage layouts: one
wave per row line for few field pairs on power-of-two sides, sixteen threads
per line otherwise), the block Hessian, the gradient and one Gauss-Newton step;
sampled checks at the 256 x 256 size; FP32 sweeps; argument errors.

The oracle computes L with a library FFT and the prior with dense circulant
matrices, the GPU with its own line FFTs, so the two share no arithmetic; they
differ by rounding only (~1e-15 per operator application, ~1e-13 after a few
hundred RK4 stages)."""
import numpy as np
import pytest

from gpu_util import Pair, colwise_relerr, need_gpu, relerr, to_dev, to_np
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu

TOL_OP = 1e-12
SMALL = inputs.bve_config(32, nsteps=12, obs_stride=8, obs_every=4, L_cells=3.0, ell=10, name='bve-32')
# ragged observation layout (48 not a multiple of the stride 5), odd window
RAGGED = inputs.bve_config(48, nsteps=9, obs_stride=5, obs_every=4, L_cells=2.5, ell=6, name='bve-48')
# grid width not a multiple of 64 (the stencils' column strips are 40 wide)
WIDE = inputs.bve_config(80, nsteps=6, obs_stride=16, obs_every=3, L_cells=3.0, ell=6, name='bve-80')
# with at most four field pairs (k <= 8) the row stages and column passes run
# one wave per line on every side (32, 48 and 80 leave lanes idle: ragged
# lines); five or more pairs take sixteen threads per line (k = 9 cases)
P64 = inputs.bve_config(64, nsteps=6, obs_stride=8, obs_every=3, L_cells=3.0, ell=6, name='bve-64')
P128 = inputs.bve_config(128, nsteps=4, obs_stride=16, obs_every=2, L_cells=3.0, ell=6, name='bve-128')
# mixed-radix wave line FFTs (4 x 4 x 4 x 3, x 5, x 2 x 3; 512 = 4^4 x 2)
P_MIXED = [inputs.bve_config(nx, nsteps=2, obs_stride=16, obs_every=1, L_cells=3.0, ell=6, name=f'bve-{nx}')
           for nx in (192, 320, 384, 512)]


@pytest.fixture(scope="module")
def small():
    need_gpu()
    return Pair(SMALL)


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("nx,k", [(32, 3), (48, 2), (64, 1), (80, 3), (96, 1), (128, 2), (160, 1), (192, 2),
                                  (256, 2), (320, 1), (384, 3), (512, 2)])
def test_inverse_laplacian_parity(nx, k):
    """Every supported side 16 B (B in {2,3,4,5,6,8,10,12,16,20,24,32}): the
    FFT path (four-step 16 x B line transforms, fields in complex pairs, odd k
    with an empty imaginary part) against the oracle's library FFT."""
    torch = need_gpu()
    from oracle import bve
    from paper_2401_15758_amd import rp4d
    cfg = inputs.bve_config(nx, nsteps=4, obs_stride=8, obs_every=2)
    p = rp4d.Problem(rp4d.Context(0), cfg)
    Z = _rand((nx * nx, k), 5)
    got = to_np(p.inv_laplacian(to_dev(Z)))
    ref = bve.inv_lap(Z.reshape(nx, nx, k)).reshape(nx * nx, k)
    assert colwise_relerr(got, ref) <= 1e-13
    got32 = to_np(p.inv_laplacian(to_dev(Z, torch.float32)))
    assert colwise_relerr(got32, ref) <= 2e-6


def test_unsupported_grid_sides_are_rejected():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx = rp4d.Context(0)
    for nx in (112, 208, 40, 1024):
        with pytest.raises(rp4d.Rp4dError) as e:
            rp4d.Problem(ctx, inputs.bve_config(nx, nsteps=4, obs_stride=8, obs_every=2))
        assert e.value.code == rp4d.EINVAL


@pytest.mark.parametrize("nx,k,L", [(32, 2, 3.0), (64, 3, 8.0), (160, 2, 8.0), (256, 1, 8.0)])
def test_prior_sqrt_parity(nx, k, L):
    need_gpu()
    from oracle import prior
    from paper_2401_15758_amd import rp4d
    cfg = inputs.bve_config(nx, nsteps=4, obs_stride=8, obs_every=2, L_cells=L)
    p = rp4d.Problem(rp4d.Context(0), cfg)
    V = _rand((nx * nx, k), 6)
    got = to_np(p.bhalf(to_dev(V)))
    ref = prior.bhalf_2d(V, nx, nx, cfg['sigma_b'], L)
    assert colwise_relerr(got, ref) <= 1e-13


@pytest.mark.parametrize("cfg", [SMALL, RAGGED, WIDE], ids=["bve-32", "bve-48-ragged", "bve-80"])
def test_fwd_observations_and_cost(cfg):
    need_gpu()
    pr = Pair(cfg, seed=2)
    obs = to_np(pr.gpu.observe(pr.traj))
    assert relerr(obs, pr.orc.observe(pr.otraj)) <= 1e-13
    d = pr.orc.innovations(pr.otraj)
    assert pr.Jobs == pytest.approx(0.5 * float(np.sum(d * d)), rel=1e-12)


@pytest.mark.parametrize("cfg,k", [(SMALL, 3), (RAGGED, 3), (WIDE, 3), (WIDE, 9), (P64, 3), (P64, 9), (P128, 1)]
                         + [(c, 2) for c in P_MIXED],
                         ids=["bve-32", "bve-48-ragged", "bve-80", "bve-80-5-pairs", "bve-64", "bve-64-5-pairs",
                              "bve-128"] + [c["name"] for c in P_MIXED])
def test_tlm_adj_hessian_parity(cfg, k):
    need_gpu()
    pr = Pair(cfg, seed=3)
    o, g = pr.orc, pr.gpu
    V = _rand((o.n, k), 7)
    Z = to_np(g.tlm(pr.traj, to_dev(V)))
    assert colwise_relerr(Z.reshape(-1, k), o.A(pr.otraj, V).reshape(-1, k)) <= TOL_OP
    W = _rand((o.n_t, o.n_obs, k), 8)
    U = to_np(g.adj(pr.traj, to_dev(W)))
    assert colwise_relerr(U, o.AT(pr.otraj, W)) <= TOL_OP
    HV = to_np(g.hessian_block(pr.traj, to_dev(V)))
    assert colwise_relerr(HV, o.hessian(pr.otraj, V)) <= TOL_OP


@pytest.mark.parametrize("cfg", [SMALL, P64], ids=["bve-32", "bve-64"])
def test_adjoint_ignores_stale_workspace(cfg):
    """The adjoint sweep's first launch sets lambda on every point and reads none
    of it (a neighbour's halo would race with those writes), so nothing clears
    lambda first: an adjoint run after another one, whose lambda is still in the
    workspace, equals the same run on a fresh problem bit for bit."""
    need_gpu()
    pr, fresh = Pair(cfg, seed=4), Pair(cfg, seed=4)
    shape = (pr.orc.n_t, pr.orc.n_obs, 2)
    _ = to_np(pr.gpu.adj(pr.traj, to_dev(_rand(shape, 20))))
    W = _rand(shape, 21)
    again = to_np(pr.gpu.adj(pr.traj, to_dev(W)))
    first = to_np(fresh.gpu.adj(fresh.traj, to_dev(W)))
    assert np.array_equal(again, first)
    assert colwise_relerr(again, pr.orc.AT(pr.otraj, W)) <= TOL_OP


def test_dot_product_identity(small):
    """<A v, w> = <v, A^T w> on the GPU alone (FP64)."""
    pr = small
    v = _rand((pr.orc.n, 1), 9)
    w = _rand((pr.orc.n_t, pr.orc.n_obs, 1), 10)
    Av = to_np(pr.gpu.tlm(pr.traj, to_dev(v)))
    ATw = to_np(pr.gpu.adj(pr.traj, to_dev(w)))
    lhs, rhs = float(np.sum(Av.reshape(-1) * w.reshape(-1))), float(np.sum(v * ATw))
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Av) * np.linalg.norm(w)


def test_gradient_parity(small):
    pr = small
    v = np.zeros(pr.orc.n)
    J, gref, _, _ = pr.orc.cost_grad(v)
    g = to_np(pr.gpu.gradient(pr.traj, to_dev(v)))
    assert relerr(g, gref) <= TOL_OP


@pytest.mark.parametrize("cfg", [SMALL, P64], ids=["bve-32", "bve-64"])
def test_fp32_sweeps_close_to_oracle(cfg):
    torch = need_gpu()
    pr = Pair(cfg, seed=2)
    V = _rand((pr.orc.n, 4), 11)
    HV = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V, torch.float32)))
    assert colwise_relerr(HV, pr.orc.hessian(pr.otraj, V)) <= 1e-4


def test_synthesis_parity():
    need_gpu()
    from oracle.problem import bve_problem
    from paper_2401_15758_amd import rp4d
    cfg = SMALL
    d = inputs.draws(cfg, seed=4)
    orc = bve_problem(cfg, d)
    p = rp4d.Problem(rp4d.Context(0), cfg)
    xb, y = p.synthesize(to_dev(d['x_true']), to_dev(d['xi']), to_dev(d['eta'].reshape(-1)))
    assert relerr(to_np(xb), orc.xb) <= 1e-14
    assert relerr(to_np(y), orc.y) <= 1e-13


@pytest.mark.parametrize("method,cfg", [("nystrom", SMALL), ("randsvd", SMALL), ("nystrom", P64)],
                         ids=["nystrom-bve-32", "randsvd-bve-32", "nystrom-bve-64"])
def test_gn_step_parity(method, cfg):
    need_gpu()
    from oracle import gn as ogn
    from paper_2401_15758_amd import rp4d
    pr = Pair(cfg, seed=5)
    ell = cfg['ell']
    Om = inputs.omega(pr.orc.n, ell, seed=1000)
    v1, dv, x1, info = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method=method, Omega=Om, rtol=1e-12)
    st = pr.gpu.gn_state()
    code = rp4d.NYSTROM if method == "nystrom" else rp4d.RANDSVD
    gi = pr.gpu.gn_step(st, sketch=code, ell=ell, omega=to_dev(Om), rtol=1e-12)
    _, gx = st.get()
    assert gi['J'] == pytest.approx(info['J'], rel=1e-12)
    assert abs(gi['pcg_iters'] - info['pcg']['iters']) <= 2
    assert relerr(to_np(st.last_step()), dv) <= 1e-10
    assert relerr(to_np(gx), x1) <= 1e-10


def test_full_size_sampled():
    """256 x 256 grid (the bve-256 grid and observation layout), 20-step window:
    observations, cost and two Hessian columns against the oracle."""
    need_gpu()
    cfg = inputs.bve_config(256, nsteps=20, obs_stride=16, obs_every=10)
    pr = Pair(cfg, seed=6)
    obs = to_np(pr.gpu.observe(pr.traj))
    assert relerr(obs, pr.orc.observe(pr.otraj)) <= 1e-13
    V = _rand((pr.orc.n, 2), 12)
    HV = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V)))
    assert colwise_relerr(HV, pr.orc.hessian(pr.otraj, V)) <= TOL_OP


def test_bad_arguments():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    ctx = rp4d.Context(0)
    with pytest.raises(rp4d.Rp4dError):
        rp4d.Problem(ctx, inputs.bve_config(40, nsteps=4, obs_every=2))      # not a multiple of 16
    with pytest.raises(rp4d.Rp4dError):
        rp4d.Problem(ctx, SMALL, ckpt_every=4)                               # 2-D stores every state
    with pytest.raises(rp4d.Rp4dError):
        rp4d.Problem(ctx, inputs.bve_config(32, nsteps=4, obs_every=2, nu=1.0))   # unstable
    p = rp4d.Problem(ctx, SMALL)
    with pytest.raises(rp4d.Rp4dError):
        rp4d.Batch(ctx, [p])                                                  # batches hold 1-D problems
    b = rp4d.Problem(ctx, inputs.CFG_SMALL)
    import torch
    with pytest.raises(rp4d.Rp4dError):
        b.inv_laplacian(torch.zeros(128, dtype=torch.float64, device="cuda"))


def test_gn_step_graph_replay_bitwise():
    """The 2-D GN step with the PCG body replayed from a captured graph equals
    the all-eager step bit for bit (10+ PCG iterations at rtol 1e-12)."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(SMALL, seed=5)
    Om = to_dev(inputs.omega(pr.orc.n, SMALL['ell'], seed=1000))
    xs, its = [], []
    for graphs in (False, True):
        pr.ctx.set_graphs(graphs)
        st = pr.gpu.gn_state()
        gi = pr.gpu.gn_step(st, sketch=rp4d.NYSTROM, ell=SMALL['ell'], omega=Om, rtol=1e-12)
        _, gx = st.get()
        torch.cuda.synchronize()
        xs.append(gx.clone())
        its.append(gi['pcg_iters'])
    pr.ctx.set_graphs(False)
    assert its[0] == its[1] and its[0] >= 5
    assert torch.equal(xs[0], xs[1])


# --- bve-256 over its whole 200-step window (the measured 2-D workload) ---
# The oracle's pieces are cached per module so that each test stays within a
# minute of host time: the trajectory, then the TLM of two columns, then their
# ADJ.

@pytest.fixture(scope="module")
def bve256():
    need_gpu()
    pr = Pair(inputs.CFG_BVE, seed=0)
    _ = pr.otraj
    return pr


@pytest.fixture(scope="module")
def bve256_tlm(bve256):
    V = _rand((bve256.orc.n, 2), 256)
    return V, bve256.orc.A(bve256.otraj, V)


def test_bve256_full_window_observations(bve256):
    pr = bve256
    obs = to_np(pr.gpu.observe(pr.traj))
    assert relerr(obs, pr.orc.observe(pr.otraj)) <= 1e-12


def test_bve256_full_window_tlm(bve256, bve256_tlm):
    """Two TLM columns over 200 steps (800 RK4 stages, one spectral Poisson
    solve per stage and column) against the oracle at 1e-12 per column."""
    pr = bve256
    V, Z = bve256_tlm
    got = to_np(pr.gpu.tlm(pr.traj, to_dev(V))).reshape(Z.shape)
    assert colwise_relerr(got.reshape(-1, 2), Z.reshape(-1, 2)) <= TOL_OP


def test_bve256_full_window_hessian(bve256, bve256_tlm):
    """(I + A^T A) V for the same two columns: 1e-12 per column."""
    pr = bve256
    V, Z = bve256_tlm
    ref = V + pr.orc.AT(pr.otraj, Z)
    HV = to_np(pr.gpu.hessian_block(pr.traj, to_dev(V)))
    assert colwise_relerr(HV, ref) <= TOL_OP
