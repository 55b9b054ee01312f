"""GPU parity of the SingleView sketch (Sec. 3.1.1, Alg. 3) with the FP64 oracle.

Both sides take the same Omega (n x l1) and Psi (m x l2); the factors are
unique only up to signs, so Lambda_hat, H_hat and the preconditioner are
compared as operators.  The oblique projector of eq. (singleviewlr) depends
only on range(Y), so the Cholesky-QR bases on the device and the Householder
bases of the oracle give the same approximation up to rounding."""
import numpy as np
import pytest

from gpu_util import Pair, colwise_relerr, need_gpu, relerr, to_dev, to_np
from oracle import gn as ogn
from oracle import sketch as osk
from paper_2401_15758_amd import inputs

pytestmark = pytest.mark.gpu

BVE_SMALL = inputs.bve_config(32, nsteps=12, obs_stride=8, obs_every=4, L_cells=3.0, ell=10, name='bve-32')


@pytest.fixture(scope="module")
def small():
    need_gpu()
    return Pair(inputs.CFG_SMALL)


def _draws(pr, l1, l2, seed):
    Om = inputs.omega(pr.orc.n, l1, seed=seed)
    Psi = np.random.default_rng(seed + 1).standard_normal((pr.orc.m, l2))
    return Om, Psi


def _probe(n, k=4, seed=7):
    return np.random.default_rng(seed).standard_normal((n, k))


def _check_parity(pr, pc, Om, Psi, tol):
    V, lam = ogn.build_precond(pr.orc, pr.otraj, 'singleview', (Om, Psi))
    glam, gnu = pc.info()
    glam = np.array(glam)
    assert gnu == 0.0 and len(glam) == len(lam)
    assert np.max(np.abs(glam - lam)) <= tol * lam[0]
    R = _probe(pr.orc.n)
    assert colwise_relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= tol
    Hh = osk.hhat_apply(to_np(pc.basis()), glam, R)
    assert colwise_relerr(Hh, osk.hhat_apply(V, lam, R)) <= 10 * tol


# (l1, l2): the paper's l2 = 2 l1 + 1 at 20 (its Burgers sketch is 15 / 31),
# odd sizes, l2 near l1, and l2 above one 64-column tile
@pytest.mark.parametrize("l1,l2", [(20, 41), (7, 15), (12, 17), (33, 67), (15, 31)])
def test_singleview_parity(small, l1, l2):
    pr = small
    Om, Psi = _draws(pr, l1, l2, seed=2000 + l1)
    pc = pr.gpu.build_precond_singleview(pr.traj, l1, l2, omega=to_dev(Om), psi=to_dev(Psi))
    _check_parity(pr, pc, Om, Psi, 1e-10)


def test_singleview_streams_are_bitwise_identical(small):
    """The co-range sweep on the side stream and on the problem stream run the
    same kernels on the same inputs: identical factors."""
    pr = small
    Om, Psi = _draws(pr, 16, 33, seed=2100)
    a = pr.gpu.build_precond_singleview(pr.traj, 16, 33, omega=to_dev(Om), psi=to_dev(Psi))
    b = pr.gpu.build_precond_singleview(pr.traj, 16, 33, omega=to_dev(Om), psi=to_dev(Psi), serial=True)
    assert np.array_equal(np.array(a.info()[0]), np.array(b.info()[0]))
    assert np.array_equal(to_np(a.basis()), to_np(b.basis()))


def test_singleview_default_l2_and_counters():
    """l2 = 0 takes min(2 l1 + 1, m); the build counts l1 offline TLM and l2
    offline ADJ columns; device draws give an effective preconditioner."""
    need_gpu()
    pr = Pair(inputs.CFG_SMALL, seed=4)
    c0 = pr.gpu.counters()
    pc = pr.gpu.build_precond_singleview(pr.traj, 15, seed=77)
    c1 = pr.gpu.counters()
    assert c1['tlm_offline'] - c0['tlm_offline'] == 15
    assert c1['adj_offline'] - c0['adj_offline'] == 31
    assert c1['sketches'] - c0['sketches'] == 1
    lam = np.array(pc.info()[0])
    assert np.all(lam >= 0) and np.all(np.diff(lam) <= 1e-12 * lam[0])
    b = to_dev(_probe(pr.orc.n, 1, seed=9)[:, 0])
    _, i0 = pr.gpu.pcg_solve(pr.traj, b, None, rtol=1e-10)
    _, i1 = pr.gpu.pcg_solve(pr.traj, b, pc, rtol=1e-10)
    assert i1["converged"] and i1["iters"] < i0["iters"]


def test_singleview_fp32_sweeps(small):
    """FP32 TLM/ADJ sweeps with FP64 post-processing stay within the FP32
    perturbation of the FP64 sketch."""
    from paper_2401_15758_amd import rp4d
    pr = small
    Om, Psi = _draws(pr, 20, 41, seed=2200)
    p64 = pr.gpu.build_precond_singleview(pr.traj, 20, 41, omega=to_dev(Om), psi=to_dev(Psi))
    p32 = pr.gpu.build_precond_singleview(pr.traj, 20, 41, omega=to_dev(Om), psi=to_dev(Psi),
                                          sketch_dtype=rp4d.F32)
    l64, l32 = np.array(p64.info()[0]), np.array(p32.info()[0])
    assert np.max(np.abs(l64 - l32)) <= 5e-3 * l64[0]
    b = to_dev(_probe(pr.orc.n, 1, seed=3)[:, 0])
    x64, i64 = pr.gpu.pcg_solve(pr.traj, b, precond=p64, rtol=1e-10)
    x32, i32 = pr.gpu.pcg_solve(pr.traj, b, precond=p32, rtol=1e-10)
    assert i32["converged"] and i32["iters"] <= i64["iters"] + 2
    assert relerr(to_np(x32), to_np(x64)) <= 1e-8


def test_singleview_bve_parity():
    """The 2-D model runs both sketches on one stream; same parity bar."""
    need_gpu()
    pr = Pair(BVE_SMALL, seed=8)
    Om, Psi = _draws(pr, 8, 17, seed=2300)
    pc = pr.gpu.build_precond_singleview(pr.traj, 8, 17, omega=to_dev(Om), psi=to_dev(Psi))
    _check_parity(pr, pc, Om, Psi, 1e-10)


def test_gn_step_singleview_parity():
    """One FP64 GN step with the SingleView preconditioner (host Omega and Psi)
    matches the oracle's step to 1e-10; counters record l1 TLM and l2 ADJ."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    Om, Psi = _draws(pr, 15, 31, seed=2400)
    st = pr.gpu.gn_state()
    gi = pr.gpu.gn_step(st, sketch=rp4d.SINGLEVIEW, ell=15, ell2=31, omega=to_dev(Om), psi=to_dev(Psi),
                        rtol=1e-12)
    _, x = st.get()
    _, dv, x1, info = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method='singleview', Omega=(Om, Psi), rtol=1e-12)
    assert relerr(to_np(st.last_step()), dv) <= 1e-10
    assert relerr(to_np(x), x1) <= 1e-10
    assert gi['J'] == pytest.approx(info['J'], rel=1e-12)
    assert abs(gi['pcg_iters'] - info['pcg']['iters']) <= 1
    assert gi['sketched'] == 1 and gi['sketch_ell'] == 15
    c = pr.gpu.counters()
    assert c['tlm_offline'] == 15 and c['adj_offline'] == 31


def test_singleview_options_are_checked(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    m = pr.orc.m
    for l1, l2 in [(0, 0), (129, 0), (20, 19), (20, m + 1)]:
        with pytest.raises(rp4d.Rp4dError) as e:
            pr.gpu.build_precond_singleview(pr.traj, l1, l2)
        assert e.value.code == rp4d.EINVAL
    with pytest.raises(rp4d.Rp4dError):
        pr.gpu.build_precond_singleview(pr.traj, 8, 17, sketch_dtype=7)


# ---------------------------------------------------------------------------
# adaptive SingleView (Sec. 3.1.2, Alg. 5)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("l1,l2,l1h,l2h,l1max,eps", [(8, 17, 8, 16, 40, 1.01), (6, 13, 5, 10, 36, 1.5),
                                                     (8, 17, 8, 16, 16, 1.01)])
def test_adaptive_singleview_parity(small, l1, l2, l1h, l2h, l1max, eps):
    """The same blocks and test vector on both sides give the same kappa_sk
    sequence, the same final sizes and the same approximation as the oracle."""
    from paper_2401_15758_amd import rp4d
    pr = small
    _, _, l2max = rp4d.sv_adaptive_sizes(pr.orc.m, l1, l1h, l1max, l2, l2h)
    Om, Psi = _draws(pr, l1max, l2max, seed=2500 + l1)
    v = inputs.omega(pr.orc.n, 1, seed=51)[:, 0]
    V, lam, kap = ogn.build_precond_singleview_adaptive(pr.orc, pr.otraj, ogn.split_blocks(Om, l1, l1h),
                                                        ogn.split_blocks(Psi, l2, l2h), v, eps)
    pc, info = pr.gpu.build_precond_singleview_adaptive(pr.traj, l1, l1h, l1max, eps_sk=eps, ell2=l2, ell2_hat=l2h,
                                                        omega=to_dev(Om), psi=to_dev(Psi), vtest=to_dev(v))
    assert info["ell"] == len(lam) and info["nkappa"] == len(kap)
    assert info["ell2"] == l2 + (len(kap) - 1) * l2h
    assert np.allclose(info["kappa"], kap, rtol=1e-9)
    glam, gnu = pc.info()
    assert gnu == 0.0
    assert np.max(np.abs(np.array(glam) - lam)) <= 1e-10 * lam[0]
    R = _probe(pr.orc.n)
    assert colwise_relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= 1e-10


@pytest.mark.parametrize("l1,l2,l1h,l2h,l1max", [(8, 17, 8, 16, 40), (6, 13, 5, 10, 36), (12, 25, 4, 8, 32)])
def test_adaptive_singleview_qr_update_parity(small, l1, l2, l1h, l2h, l1max):
    """With the QR update of Alg. 6 (wide A2 B1 when l2_hat < l1) the device
    matches the oracle's Alg. 6 run (qr='update'), which equals refactoring M."""
    from paper_2401_15758_amd import rp4d
    pr = small
    _, _, l2max = rp4d.sv_adaptive_sizes(pr.orc.m, l1, l1h, l1max, l2, l2h)
    Om, Psi = _draws(pr, l1max, l2max, seed=2700 + l1)
    v = inputs.omega(pr.orc.n, 1, seed=53)[:, 0]
    m = pr.orc.m
    A = lambda X: pr.orc.A(pr.otraj, X).reshape(m, -1)
    AT = lambda W: pr.orc.AT(pr.otraj, W.reshape(pr.orc.n_t, pr.orc.n_obs, -1))
    H = lambda X: pr.orc.misfit_hessian(pr.otraj, X)
    V, lam, kap = osk.singleview_adaptive(A, AT, H, ogn.split_blocks(Om, l1, l1h), ogn.split_blocks(Psi, l2, l2h),
                                          v, 0.5, qr='update')
    pc, info = pr.gpu.build_precond_singleview_adaptive(pr.traj, l1, l1h, l1max, eps_sk=0.5, ell2=l2, ell2_hat=l2h,
                                                        omega=to_dev(Om), psi=to_dev(Psi), vtest=to_dev(v),
                                                        qr_update=True)
    assert info["ell"] == len(lam) == l1max - (l1max - l1) % l1h and info["nkappa"] == len(kap)
    assert np.allclose(info["kappa"], kap, rtol=1e-9)
    glam, _ = pc.info()
    assert np.max(np.abs(np.array(glam) - lam)) <= 1e-10 * lam[0]
    R = _probe(pr.orc.n)
    assert colwise_relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= 1e-10


def test_adaptive_singleview_streams_are_bitwise_identical(small):
    pr = small
    a, ia = pr.gpu.build_precond_singleview_adaptive(pr.traj, 8, 8, 32, eps_sk=1.0, seed=31)
    b, ib = pr.gpu.build_precond_singleview_adaptive(pr.traj, 8, 8, 32, eps_sk=1.0, seed=31, serial=True)
    assert ia["kappa"] == ib["kappa"] and ia["ell"] == ib["ell"] == 32
    assert np.array_equal(to_np(a.basis()), to_np(b.basis()))


def test_adaptive_singleview_device_draws_stop_at_tolerance():
    """With device draws the loop ends at the first kappa_sk <= eps_sk (or at
    l1_max); the counters record every column and every kappa_sk product."""
    need_gpu()
    pr = Pair(inputs.CFG_SMALL, seed=6)
    c0 = pr.gpu.counters()
    pc, info = pr.gpu.build_precond_singleview_adaptive(pr.traj, 4, 4, 48, eps_sk=1.05, seed=99)
    c1 = pr.gpu.counters()
    k = info["kappa"]
    assert k[-1] <= 1.05 or info["ell"] + 4 > 48
    assert all(x > 1.05 for x in k[:-1])
    assert info["ell"] == 4 + 4 * (info["nkappa"] - 1)
    assert c1["tlm_offline"] - c0["tlm_offline"] == info["ell"] + info["nkappa"]
    assert c1["adj_offline"] - c0["adj_offline"] == info["ell2"] + info["nkappa"]
    b = to_dev(_probe(pr.orc.n, 1, seed=9)[:, 0])
    _, i0 = pr.gpu.pcg_solve(pr.traj, b, None, rtol=1e-10)
    _, i1 = pr.gpu.pcg_solve(pr.traj, b, pc, rtol=1e-10)
    assert i1["converged"] and i1["iters"] < i0["iters"]


def test_gn_step_adaptive_singleview_parity():
    """A GN step with the adaptive SingleView preconditioner (host blocks and
    test vector) matches the oracle's step to 1e-10."""
    need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL)
    l1, l1h, l1max, l2, l2h = 8, 8, 40, 17, 16
    _, _, l2max = rp4d.sv_adaptive_sizes(pr.orc.m, l1, l1h, l1max, l2, l2h)
    Om, Psi = _draws(pr, l1max, l2max, seed=2600)
    vh = inputs.omega(pr.orc.n, 1, seed=811)[:, 0]
    st = pr.gpu.gn_state()
    gi = pr.gpu.gn_step(st, sketch=rp4d.SINGLEVIEW_ADAPTIVE, ell=l1, ell_hat=l1h, ell_max=l1max, ell2=l2,
                        ell2_hat=l2h, eps_sk=1.01, omega=to_dev(Om), psi=to_dev(Psi), vhat=to_dev(vh), rtol=1e-12)
    _, x = st.get()
    _, _, x1, oinf = ogn.gn_step(pr.orc, np.zeros(pr.orc.n), method='singleview_adaptive', Omega=(Om, Psi),
                                 vhat=vh, rtol=1e-12,
                                 adaptive=dict(ell0=l1, ell_hat=l1h, ell2=l2, ell2_hat=l2h, eps_sk=1.01))
    assert relerr(to_np(x), x1) <= 1e-10
    assert gi["sketch_ell"] == oinf["precond"][0].shape[1]
    assert 0 < gi["kappa_sk"]
    assert abs(gi["pcg_iters"] - oinf["pcg"]["iters"]) <= 1


def test_adaptive_singleview_options_are_checked(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    m = pr.orc.m
    bad = [dict(ell1=0, ell1_hat=4, ell1_max=16), dict(ell1=8, ell1_hat=0, ell1_max=16),
           dict(ell1=8, ell1_hat=4, ell1_max=4), dict(ell1=8, ell1_hat=4, ell1_max=200),
           dict(ell1=8, ell1_hat=4, ell1_max=16, ell2=7), dict(ell1=8, ell1_hat=4, ell1_max=16, ell2_hat=3),
           dict(ell1=8, ell1_hat=8, ell1_max=64, ell2=17, ell2_hat=m)]
    for kw in bad:
        with pytest.raises(rp4d.Rp4dError) as e:
            pr.gpu.build_precond_singleview_adaptive(pr.traj, eps_sk=1.01, **kw)
        assert e.value.code == rp4d.EINVAL
    with pytest.raises(rp4d.Rp4dError):
        pr.gpu.build_precond_singleview_adaptive(pr.traj, 8, 4, 16, eps_sk=0.0)
