"""GPU parity of the sketches (Nystrom Alg. 2, RandSVD Alg. 1), the limited-memory
preconditioner, PCG, the reuse test and the Gauss-Newton step with the FP64 oracle.

Sketch factors are unique only up to sign/rotation, so operators are compared:
Lambda_hat (sorted), H_hat and P applied to probes.  The FP64 GN step is
compared at PCG rtol 1e-12 (two correct CG runs at rtol 1e-6 may differ by
~kappa 1e-6, which is not a parity statement)."""
import numpy as np
import pytest

from gpu_util import Pair, colwise_relerr, need_gpu, relerr, to_dev, to_np
from oracle import gn as ogn
from oracle import sketch as osk
from oracle.pcg import pcg as opcg
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu

TOL_GN = 1e-10   # FP64 GN step, relative


@pytest.fixture(scope="module")
def small():
    need_gpu()
    return Pair(inputs.CFG_SMALL)


def _probe(n, k=4, seed=7):
    return np.random.default_rng(seed).standard_normal((n, k))


@pytest.mark.parametrize("method,ell", [("nystrom", 20), ("randsvd", 20), ("nystrom", 7), ("randsvd", 7),
                                        ("nystrom", 33), ("randsvd", 33), ("nystrom", 64)])
def test_sketch_parity(small, method, ell):
    from paper_2401_15758_amd import rp4d
    pr = small
    Om = inputs.omega(pr.orc.n, ell, seed=1000 + ell)
    V, lam = ogn.build_precond(pr.orc, pr.otraj, method, Om)
    code = rp4d.NYSTROM if method == "nystrom" else rp4d.RANDSVD
    pc = pr.gpu.build_precond(pr.traj, code, ell, omega=to_dev(Om))
    glam, gnu = pc.info()
    glam = np.array(glam)
    assert np.max(np.abs(glam - lam)) <= 1e-10 * lam[0]
    if method == "nystrom":
        Y0 = pr.orc.misfit_hessian(pr.otraj, Om)
        nu = np.sqrt(pr.orc.n) * 2.0 ** -52 * np.linalg.norm(Y0, 2)
        assert gnu == pytest.approx(nu, rel=1e-12)
    R = _probe(pr.orc.n)
    PR = to_np(pc.apply(to_dev(R)))
    assert colwise_relerr(PR, osk.lmp_apply(V, lam, R)) <= 1e-10
    Vg = to_np(pc.basis())
    Hh = osk.hhat_apply(Vg, glam, R)
    assert colwise_relerr(Hh, osk.hhat_apply(V, lam, R)) <= 1e-9


@pytest.mark.parametrize("ell0,ell_hat,ell_max,eps", [(8, 8, 40, 1.01), (6, 5, 36, 1.5), (8, 8, 16, 1.01)])
def test_adaptive_randsvd_parity(small, ell0, ell_hat, ell_max, eps):
    """Adaptive RandSVD (Alg. 4): the same Gaussian blocks and test vector on
    both sides give the same sequence of kappa_sk, the same final size and the
    same approximation as the oracle."""
    pr = small
    Om = inputs.omega(pr.orc.n, ell_max, seed=700 + ell0)
    v = inputs.omega(pr.orc.n, 1, seed=50)[:, 0]
    blocks = [Om[:, :ell0]] + [Om[:, c:c + ell_hat] for c in range(ell0, ell_max - ell_hat + 1, ell_hat)]
    V, lam, kap = ogn.build_precond_adaptive(pr.orc, pr.otraj, blocks, v, eps)
    pc, info = pr.gpu.build_precond_adaptive(pr.traj, ell0, ell_hat, ell_max, eps_sk=eps, omega=to_dev(Om),
                                             vtest=to_dev(v))
    assert info["ell"] == len(lam) and info["nkappa"] == len(kap)
    assert np.allclose(info["kappa"], kap, rtol=1e-9)
    glam, gnu = pc.info()
    assert gnu == 0.0
    assert np.max(np.abs(np.array(glam) - lam)) <= 1e-10 * lam[0]
    R = _probe(pr.orc.n)
    assert colwise_relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= 1e-10


def test_adaptive_randsvd_device_draws_stop_at_tolerance(small):
    """With device draws the loop ends once kappa_sk <= eps_sk (or at ell_max),
    and the resulting preconditioner cuts the PCG iterations."""
    from paper_2401_15758_amd import rp4d
    pr = small
    pc, info = pr.gpu.build_precond_adaptive(pr.traj, 4, 4, 64, eps_sk=1.05, seed=99)
    k = info["kappa"]
    assert k[-1] <= 1.05 or info["ell"] + 4 > 64
    assert all(x > 1.05 for x in k[:-1])
    assert info["ell"] == 4 + 4 * (info["nkappa"] - 1)
    b = to_dev(_probe(pr.orc.n, 1, seed=9)[:, 0])
    _, i0 = pr.gpu.pcg_solve(pr.traj, b, None, rtol=1e-10)
    _, i1 = pr.gpu.pcg_solve(pr.traj, b, pc, rtol=1e-10)
    assert i1["iters"] < i0["iters"]


def test_gn_step_adaptive_parity():
    """A GN step with the adaptive RandSVD preconditioner (host blocks and test
    vector) matches the oracle's GN step to 1e-10."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    Om = inputs.omega(pr.orc.n, 40, seed=810)
    vh = inputs.omega(pr.orc.n, 1, seed=811)[:, 0]
    st = pr.gpu.gn_state()
    info = pr.gpu.gn_step(st, sketch=rp4d.RANDSVD_ADAPTIVE, ell=8, ell_hat=8, ell_max=40, eps_sk=1.01,
                          omega=to_dev(Om), vhat=to_dev(vh), rtol=1e-12)
    _, x = st.get()
    _, _, x1, oinf = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method='randsvd_adaptive', Omega=Om, vhat=vh,
                                 rtol=1e-12, adaptive=dict(ell0=8, ell_hat=8, eps_sk=1.01))
    assert relerr(to_np(x), x1) <= 1e-10
    assert info["sketch_ell"] == oinf["precond"][0].shape[1]
    assert 0 < info["kappa_sk"] <= 1.01
    assert info["pcg_iters"] == oinf["pcg"]["iters"]


def test_adaptive_options_are_checked(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    for args in [(0, 4, 16), (8, 0, 16), (8, 4, 4), (8, 4, 200)]:
        with pytest.raises(rp4d.Rp4dError):
            pr.gpu.build_precond_adaptive(pr.traj, *args, eps_sk=1.01)
    with pytest.raises(rp4d.Rp4dError):
        pr.gpu.build_precond_adaptive(pr.traj, 8, 4, 16, eps_sk=0.0)


def test_randsvd_rank_deficient_sketch_is_reported(small):
    """64 columns exceed the numerical rank of A on the 128-point problem: the
    thin QR of Y = A Omega by Cholesky QR (shifted CholeskyQR3 included) cannot
    orthonormalise it, and the build reports ENOTSPD instead of a wrong basis."""
    from paper_2401_15758_amd import rp4d
    pr = small
    Om = inputs.omega(pr.orc.n, 64, seed=1064)
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.build_precond(pr.traj, rp4d.RANDSVD, 64, omega=to_dev(Om))
    assert e.value.code == rp4d.ENOTSPD


def test_precond_inverts_one_plus_hhat(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    pc = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 20, omega=to_dev(inputs.omega(pr.orc.n, 20)))
    Vg = to_np(pc.basis())
    lam = np.array(pc.info()[0])
    R = _probe(pr.orc.n)
    M = R + osk.hhat_apply(Vg, lam, R)            # (I + H_hat) R
    back = to_np(pc.apply(to_dev(M)))
    assert colwise_relerr(back, R) <= 1e-10


def test_philox_sketch_statistics(small):
    """Device-drawn Omega: moments of Philox4x32-10 + Box-Muller normals."""
    torch = need_gpu()
    pr = small
    out = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    pr.ctx.philox_normal(1234, out.numel(), out)
    x = to_np(out)
    assert abs(x.mean()) < 5e-3 and abs(x.var() - 1) < 5e-3
    assert abs(np.mean(x ** 4) - 3) < 3e-2
    from scipy import stats
    assert stats.kstest(x[:200000], 'norm').pvalue > 1e-4
    y = to_np(pr.ctx.philox_normal(1234, out.numel(), torch.empty_like(out)))
    assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", [None, "nystrom"])
def test_pcg_parity(small, prec):
    from paper_2401_15758_amd import rp4d
    pr = small
    b = np.random.default_rng(3).standard_normal(pr.orc.n)
    P = None
    pc = None
    if prec:
        Om = inputs.omega(pr.orc.n, 20)
        P = ogn.build_precond(pr.orc, pr.otraj, prec, Om)
        pc = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 20, omega=to_dev(Om))
    xr, ir = opcg(lambda v: pr.orc.hessian(pr.otraj, v), b,
                  prec=(lambda r: osk.lmp_apply(P[0], P[1], r)) if P else None, rtol=1e-12)
    x, info = pr.gpu.pcg_solve(pr.traj, to_dev(b), precond=pc, rtol=1e-12)
    x = to_np(x)
    assert info['converged'] and abs(info['iters'] - ir['iters']) <= 1
    assert relerr(x, xr) <= TOL_GN
    assert info['true_relres'] <= 1e-10


def test_pcg_noconv_keeps_iterate(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    b = to_dev(np.ones(pr.orc.n))
    x, info = pr.gpu.pcg_solve(pr.traj, b, rtol=1e-14, maxit=2, raise_noconv=False)
    assert info['iters'] == 2 and not info['converged']
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.pcg_solve(pr.traj, b, rtol=1e-14, maxit=1)
    assert e.value.code == rp4d.ENOCONV


def test_pcg_zero_rhs(small):
    """b = 0: x = 0 after no iteration, whatever x held.  The first iteration,
    enqueued before |b| is read, is discarded and not counted; the one product
    counted is pcg_solve's true-residual check."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = small
    pc12 = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 12, omega=to_dev(inputs.omega(pr.orc.n, 12)))
    for pc in (None, pc12):
        b = torch.zeros(pr.orc.n, dtype=torch.float64, device="cuda")
        x = torch.full_like(b, float("nan"))
        before = pr.gpu.counters()
        x, info = pr.gpu.pcg_solve(pr.traj, b, precond=pc, rtol=1e-10, x=x)
        after = pr.gpu.counters()
        assert info['iters'] == 0 and info['converged'] and info['relres'] == 0.0
        assert torch.count_nonzero(x).item() == 0
        assert info['true_relres'] == 0.0
        assert after['hv_columns'] == before['hv_columns'] + 1 and after['tlm_online'] == before['tlm_online']


def test_kappa_re_parity(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    Om = inputs.omega(pr.orc.n, 10)
    V, lam = ogn.build_precond(pr.orc, pr.otraj, "nystrom", Om)
    pc = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 10, omega=to_dev(Om))
    vh = inputs.unit_vector(pr.orc.n)
    k = pr.gpu.kappa_re(pr.traj, pc, to_dev(vh))
    assert k == pytest.approx(ogn.kappa_re(pr.orc, pr.otraj, V, lam, vh), rel=1e-10)


@pytest.mark.parametrize("method", ["nystrom", "randsvd", "none"])
def test_gn_step_parity(method):
    """One FP64 GN step on burgers-128: dv and x+ within 1e-10 of the oracle."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    ell = 20
    Om = inputs.omega(pr.orc.n, ell, seed=1000)
    v0 = np.zeros(pr.orc.n)
    v1, dv, x1, info = ogn.gn_step(pr.orc, v0, method=method, Omega=Om, rtol=1e-12)
    st = pr.gpu.gn_state()
    code = dict(nystrom=rp4d.NYSTROM, randsvd=rp4d.RANDSVD, none=rp4d.NOPREC)[method]
    gi = pr.gpu.gn_step(st, sketch=code, ell=ell, omega=to_dev(Om), rtol=1e-12)
    gdv = to_np(st.last_step())
    gv, gx = st.get()
    assert gi['J'] == pytest.approx(info['J'], rel=1e-12)
    assert gi['gnorm_inf'] == pytest.approx(info['gnorm_inf'], rel=1e-11)
    assert abs(gi['pcg_iters'] - info['pcg']['iters']) <= 1
    assert relerr(gdv, dv) <= TOL_GN
    assert relerr(to_np(gx), x1) <= TOL_GN
    c = pr.gpu.counters()
    assert c['fwd'] == 2            # data check at construction + the step
    assert c['tlm_online'] == gi['pcg_iters'] and c['adj_online'] == gi['pcg_iters'] + 1
    if method != "none":
        assert c['tlm_offline'] == c['adj_offline'] == ell and c['sketches'] == 1


def test_three_gn_steps_with_reuse_test():
    """Three GN steps with the kappa_re reuse test: J decreases, the reuse
    decision matches the oracle's, and iterates stay within 1e-10."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    ell, eps_re = 20, 10.0
    v = np.zeros(pr.orc.n)
    st = pr.gpu.gn_state()
    P = None
    vh = inputs.unit_vector(pr.orc.n, seed=77)
    for k in range(3):
        Om = inputs.omega(pr.orc.n, ell, seed=2000 + k)
        v, dv, x, info = ogn.gn_step(pr.orc, v, method='nystrom', Omega=Om, rtol=1e-12, precond=P,
                                     reuse_eps=eps_re, vhat=vh)
        P = info['precond']
        gi = pr.gpu.gn_step(st, sketch=rp4d.NYSTROM, ell=ell, omega=to_dev(Om), rtol=1e-12, reuse_eps=eps_re,
                            vhat=to_dev(vh))
        assert gi['reused'] == int(info['reused'])
        if info['kappa_re'] is not None:
            assert gi['kappa_re'] == pytest.approx(info['kappa_re'], rel=1e-8)
        gv, gx = st.get()
        assert relerr(to_np(gv), v) <= TOL_GN
        assert relerr(to_np(gx), x) <= TOL_GN


def test_fp32_sketch_then_fp64_pcg(small):
    """Mixed precision: FP32 sketch sweeps, FP64 post-processing and PCG; the solve
    still meets its FP64 tolerance and the preconditioner stays effective."""
    from paper_2401_15758_amd import rp4d
    pr = small
    b = np.random.default_rng(9).standard_normal(pr.orc.n)
    Om = to_dev(inputs.omega(pr.orc.n, 20))
    p64 = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 20, omega=Om)
    p32 = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 20, omega=Om, sketch_dtype=rp4d.F32)
    l64, l32 = np.array(p64.info()[0]), np.array(p32.info()[0])
    # FP32 sweeps perturb H Omega by ~1e-4 relative; the sketch eigenvalues move by ~1e-3 of the largest
    assert np.max(np.abs(l64 - l32)) <= 5e-3 * l64[0]
    x64, i64 = pr.gpu.pcg_solve(pr.traj, to_dev(b), precond=p64, rtol=1e-10)
    x32, i32 = pr.gpu.pcg_solve(pr.traj, to_dev(b), precond=p32, rtol=1e-10)
    assert i32['converged'] and i32['iters'] <= i64['iters'] + 2
    assert relerr(to_np(x32), to_np(x64)) <= 1e-8


@pytest.mark.parametrize("use_prec", [False, True])
def test_pcg_graph_replay_is_bitwise_eager(small, use_prec):
    """PCG iterations after the second replay a captured HIP graph of the
    iteration body; every replay is followed by the eager residual read-back,
    and the solution must equal the all-eager solve bit for bit."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = small
    pc = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 7, omega=to_dev(inputs.omega(pr.orc.n, 7))) if use_prec else None
    b = to_dev(_probe(pr.orc.n, 1, seed=31)[:, 0])
    out = {}
    for graphs in (False, True):
        pr.ctx.set_graphs(graphs)
        x, info = pr.gpu.pcg_solve(pr.traj, b, precond=pc, rtol=1e-11)
        torch.cuda.synchronize()
        out[graphs] = (x.clone(), info['iters'])
    pr.ctx.set_graphs(False)
    assert out[True][1] == out[False][1] and out[True][1] >= 5
    assert torch.equal(out[True][0], out[False][0])


@pytest.mark.parametrize("method", ["nystrom", "randsvd", "singleview"])
def test_gn_step_sketchsolv_parity(method):
    """SketchSolv (Sec. 3.2.1, eq. (dxsol)): the direction is one application of
    eq. (woodbury) to -g_v, no PCG; dv and x+ within 1e-10 of the oracle."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    ell = 20
    Om = inputs.omega(pr.orc.n, ell, seed=1300)
    Psi = np.random.default_rng(1301).standard_normal((pr.orc.m, 2 * ell + 1))
    arg = (Om, Psi) if method == "singleview" else Om
    _, dv, x1, info = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method=method, Omega=arg, solve='sketch')
    code = dict(nystrom=rp4d.NYSTROM, randsvd=rp4d.RANDSVD, singleview=rp4d.SINGLEVIEW)[method]
    st = pr.gpu.gn_state()
    gi = pr.gpu.gn_step(st, sketch=code, ell=ell, omega=to_dev(Om),
                        psi=to_dev(Psi) if method == "singleview" else None, solve=rp4d.SOLVE_SKETCH)
    _, gx = st.get()
    assert gi['pcg_iters'] == 0 and gi['pcg_converged'] == 1 and gi['pcg_relres'] == -1.0
    assert gi['J'] == pytest.approx(info['J'], rel=1e-12)
    assert gi['gnorm_inf'] == pytest.approx(info['gnorm_inf'], rel=1e-11)
    assert relerr(to_np(st.last_step()), dv) <= TOL_GN
    assert relerr(to_np(gx), x1) <= TOL_GN
    c = pr.gpu.counters()
    assert c['tlm_online'] == 0 and c['adj_online'] == 1


def test_sketchsolv_requires_a_sketch():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    st = pr.gpu.gn_state()
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.gn_step(st, sketch=rp4d.NOPREC, solve=rp4d.SOLVE_SKETCH)
    assert e.value.code == rp4d.EINVAL


@pytest.mark.parametrize("ell0,ell_hat,ell_max,eps", [(8, 8, 40, 1.01), (6, 5, 36, 1.5), (8, 8, 16, 1.01)])
def test_adaptive_nystrom_parity(small, ell0, ell_hat, ell_max, eps):
    """Adaptive Nystrom: the same blocks and test vector give the same kappa_sk
    sequence, final size, shift and approximation as the oracle."""
    from paper_2401_15758_amd import rp4d
    pr = small
    Om = inputs.omega(pr.orc.n, ell_max, seed=900 + ell0)
    v = inputs.omega(pr.orc.n, 1, seed=52)[:, 0]
    V, lam, nu, kap = ogn.build_precond_nystrom_adaptive(pr.orc, pr.otraj, ogn.split_blocks(Om, ell0, ell_hat), v, eps)
    pc, info = pr.gpu.build_precond_adaptive(pr.traj, ell0, ell_hat, ell_max, eps_sk=eps, omega=to_dev(Om),
                                             vtest=to_dev(v), method=rp4d.NYSTROM)
    assert info["ell"] == len(lam) and info["nkappa"] == len(kap)
    assert np.allclose(info["kappa"], kap, rtol=1e-9)
    glam, gnu = pc.info()
    assert gnu == pytest.approx(nu, rel=1e-12)
    assert np.max(np.abs(np.array(glam) - lam)) <= 1e-10 * lam[0]
    R = _probe(pr.orc.n)
    assert colwise_relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= 1e-10


def test_adaptive_nystrom_device_draws_stop_at_tolerance():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL, seed=9)
    c0 = pr.gpu.counters()
    pc, info = pr.gpu.build_precond_adaptive(pr.traj, 4, 4, 64, eps_sk=1.05, seed=123, method=rp4d.NYSTROM)
    c1 = pr.gpu.counters()
    k = info["kappa"]
    assert k[-1] <= 1.05 or info["ell"] + 4 > 64
    assert all(x > 1.05 for x in k[:-1])
    assert c1["tlm_offline"] - c0["tlm_offline"] == info["ell"] + info["nkappa"]
    b = to_dev(_probe(pr.orc.n, 1, seed=9)[:, 0])
    _, i0 = pr.gpu.pcg_solve(pr.traj, b, None, rtol=1e-10)
    _, i1 = pr.gpu.pcg_solve(pr.traj, b, pc, rtol=1e-10)
    assert i1["iters"] < i0["iters"]


def test_gn_step_adaptive_nystrom_parity():
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    Om = inputs.omega(pr.orc.n, 40, seed=910)
    vh = inputs.omega(pr.orc.n, 1, seed=911)[:, 0]
    st = pr.gpu.gn_state()
    info = pr.gpu.gn_step(st, sketch=rp4d.NYSTROM_ADAPTIVE, ell=8, ell_hat=8, ell_max=40, eps_sk=1.01,
                          omega=to_dev(Om), vhat=to_dev(vh), rtol=1e-12)
    _, x = st.get()
    _, _, x1, oinf = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method='nystrom_adaptive', Omega=Om, vhat=vh,
                                 rtol=1e-12, adaptive=dict(ell0=8, ell_hat=8, eps_sk=1.01))
    assert relerr(to_np(x), x1) <= 1e-10
    assert info["sketch_ell"] == oinf["precond"][0].shape[1]
    assert abs(info["pcg_iters"] - oinf["pcg"]["iters"]) <= 1


@pytest.mark.parametrize("which,ell,solve,alpha,trials", [("wall", 2, "sketch", 0.25, 3),
                                                         ("periodic", 20, "pcg", 1.0, 1),
                                                         ("periodic", 2, "sketch", None, None)])
def test_gn_step_line_search_parity(which, ell, solve, alpha, trials):
    """Armijo backtracking: the same step length and trial count as the oracle
    and the same iterate to 1e-10.  The last case (SketchSolv with a 2-column
    sketch on burgers-128) first tries steps whose trajectories overflow, which
    count as failed trials on both sides."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    cfg = inputs.CFG_WALL_SMALL if which == "wall" else inputs.CFG_SMALL
    pr = Pair(cfg, seed=0)
    Om = inputs.omega(pr.orc.n, ell, seed=1000)
    _, _, x1, info = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method='nystrom', Omega=Om, rtol=1e-12,
                                 solve=solve, line_search=True)
    if alpha is not None:
        assert info['alpha'] == alpha and info['ls_trials'] == trials
    st = pr.gpu.gn_state()
    c0 = pr.gpu.counters()
    gi = pr.gpu.gn_step(st, sketch=rp4d.NYSTROM, ell=ell, omega=to_dev(Om), rtol=1e-12, line_search=True,
                        solve=rp4d.SOLVE_SKETCH if solve == "sketch" else rp4d.SOLVE_PCG)
    c1 = pr.gpu.counters()
    assert gi['alpha'] == info['alpha'] and gi['ls_trials'] == info['ls_trials']
    assert c1['fwd'] - c0['fwd'] == 1 + gi['ls_trials']
    _, gx = st.get()
    assert relerr(to_np(gx), x1) <= 1e-10


MED = inputs.burgers_config(512, 100, 4, 10, dt_cfg=1e-3, L_b=0.01, ell=128, name='burgers-512')  # rank(A) > 128


@pytest.mark.parametrize("method", ["nystrom", "randsvd"])
def test_sketch_parity_at_the_largest_size(method):
    """l = 128, the largest sketch (the order-128 Cholesky, triangular inverse
    and Jacobi kernels, Gram tiles beyond 64 columns) on a 512-point problem
    with m = 1280 observations."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(MED, seed=2)
    Om = inputs.omega(pr.orc.n, 128, seed=1128)
    V, lam = ogn.build_precond(pr.orc, pr.otraj, method, Om)
    pc = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM if method == "nystrom" else rp4d.RANDSVD, 128,
                              omega=to_dev(Om))
    glam = np.array(pc.info()[0])
    assert np.max(np.abs(glam - lam)) <= 1e-10 * lam[0]
    R = _probe(pr.orc.n)
    assert colwise_relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= 1e-10


@pytest.mark.parametrize("method", ["nystrom", "randsvd"])
def test_gn_step_exact_and_factored_preconditioners_agree(method):
    """SketchPrec with the eigen-decomposed preconditioner (exact_lmp) and with
    the factored form (the default) reach the oracle's step to 1e-10.  The two
    operators differ by at most the Nystrom shift nu in norm (the factored form
    keeps the shift), so at rtol 1e-12, the attainable accuracy, their PCG
    iteration counts may differ by one, and from the oracle's by one."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    Om = inputs.omega(pr.orc.n, 12, seed=1400)
    _, dv, x1, info = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method=method, Omega=Om, rtol=1e-12)
    code = rp4d.NYSTROM if method == "nystrom" else rp4d.RANDSVD
    its = []
    for exact in (True, False):
        st = pr.gpu.gn_state()
        gi = pr.gpu.gn_step(st, sketch=code, ell=12, omega=to_dev(Om), rtol=1e-12, exact_lmp=exact)
        _, gx = st.get()
        assert relerr(to_np(st.last_step()), dv) <= TOL_GN
        assert relerr(to_np(gx), x1) <= TOL_GN
        its.append(gi['pcg_iters'])
    # rtol 1e-12 is near the attainable accuracy: the two forms may differ by one iteration
    assert abs(its[0] - its[1]) <= 1 and abs(its[0] - info['pcg']['iters']) <= 1


def test_objects_can_be_destroyed_in_any_order():
    """Destruction reads nothing outside the object: a context, problem,
    trajectory, preconditioner and GN state closed owner-first (as a language
    runtime's finaliser may do at exit) release cleanly."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    pc = pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 8, seed=3)
    st = pr.gpu.gn_state()
    pr.gpu.gn_step(st, sketch=rp4d.NYSTROM, ell=8, seed=4)
    pr.ctx.close()
    pr.gpu.close()
    pr.traj.close()
    pc.close()
    st.close()
    torch.cuda.synchronize()


def test_pipelined_gn_steps_match_sequential():
    """burgers-4096: with every row stored, a Nystrom or RandSVD GN step runs its
    FWD on the side stream and the sketch's TLM sweep follows it launch by launch;
    with checkpointing (ckpt_every = 10) the two run one after the other.  The
    checkpointed trajectory is bitwise the stored one, so the iterates of three
    Nystrom steps (and one RandSVD step) agree bit for bit -- also with the FWD
    cut into two-step launches, which makes the TLM wait on many more events, and
    with the committed tuned tilings."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    cfg = inputs.CFG_LARGE
    d = inputs.draws(cfg, seed=0)
    ctx = rp4d.Context(0)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")

    def run(ckpt, sketch, steps, short_fwd=False, tuned=False):
        prob = rp4d.Problem(ctx, cfg, ckpt_every=ckpt)
        xb, y = prob.synthesize(dev(d["x_true"]), dev(d["xi"]), dev(d["eta"].reshape(-1)))
        prob.set_data(xb, y.reshape(-1))
        if tuned:  # the committed tilings (sweeps and FWD with different steps per launch)
            from paper_2401_15758_amd import autotune
            for k in (64, 1):
                autotune.apply_cached(prob, cfg["nsteps"], k)
        if short_fwd:
            prob.set_sweep_tiling(mode=rp4d.MODE_FWD, ppt=2, threads=64, tile=96, steps=2, xch=rp4d.XCH_WAVE)
        st = prob.gn_state()
        infos = [prob.gn_step(st, sketch=sketch, ell=64, seed=500 + i, rtol=1e-8) for i in range(steps)]
        v, x = st.get()
        torch.cuda.synchronize()
        return [(i["J"], i["pcg_iters"], i["gnorm_inf"]) for i in infos], v.clone(), x.clone()

    for sketch, steps in ((rp4d.NYSTROM, 3), (rp4d.RANDSVD, 1)):
        ref = run(10, sketch, steps)
        for short, tuned in ((False, False), (True, False), (False, True)):
            got = run(0, sketch, steps, short_fwd=short, tuned=tuned)
            assert got[0] == ref[0], (sketch, short, tuned)
            assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2]), (sketch, short, tuned)


@pytest.mark.parametrize("method", ["nystrom", "randsvd"])
def test_bf16_gram_option(small, method):
    """The BF16 Gram option of the sketch post-processing: Lambda_hat within the
    bfloat16 rounding scale of the FP64 build (Weyl: the eigenvalues move by at
    most the Gram's perturbation, here entries off by O(2^-8) of their
    Cauchy-Schwarz bound), and PCG with that preconditioner still meets a
    1e-10 residual against the oracle's solution.  Other dtypes are rejected."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = small
    m = rp4d.NYSTROM if method == "nystrom" else rp4d.RANDSVD
    om = to_dev(inputs.omega(pr.orc.n, 20))
    lam64 = np.array(pr.gpu.build_precond(pr.traj, m, 20, omega=om).info()[0])
    pr.ctx.set_gram_precision(rp4d.BF16)
    try:
        pc = pr.gpu.build_precond(pr.traj, m, 20, omega=om)
        lam16 = np.array(pc.info()[0])
        b = _probe(pr.orc.n, 1, seed=41)[:, 0]
        x, info = pr.gpu.pcg_solve(pr.traj, to_dev(b), precond=pc, rtol=1e-12)
    finally:
        pr.ctx.set_gram_precision(rp4d.F64)
    assert np.max(np.abs(lam16 - lam64)) <= 2.0 ** -6 * lam64.max()
    assert np.max(np.abs(lam16 - lam64)) > 0          # the option changed the arithmetic
    xo = np.linalg.solve(pr.orc.hessian(pr.otraj, np.eye(pr.orc.n)), b)   # the oracle's (I + H)
    assert relerr(to_np(x), xo) <= 1e-10
    with pytest.raises(rp4d.Rp4dError):
        pr.ctx.set_gram_precision(rp4d.F32)
