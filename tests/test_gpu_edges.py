"""GPU edge cases and failure paths, each against the oracle: Nystrom's shift
retries (Alg. 2; x10 per retry, at most three) on a caller-supplied indefinite
sketch, the ENOTSPD exits, PCG with a tolerance x_0 = 0 already meets, non-finite
data reported as ENONFINITE, a GN step that fails mid-sketch, and the device's
Philox stream against the oracle's."""
import numpy as np
import pytest

from gpu_util import Pair, need_gpu, relerr, to_dev, to_np
from oracle import gn as ogn
from oracle import rng as orng
from oracle import sketch as osk
from oracle.pcg import pcg as opcg
from paper_2401_15758_amd import inputs
from test_oracle_sketch import _indefinite_sketch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    need_gpu()
    return Pair(inputs.CFG_SMALL)


@pytest.mark.parametrize("ratio, retries", [(3.0, 1), (30.0, 2), (300.0, 3)])
def test_nystrom_shift_retries_match_oracle(small, ratio, retries):
    """n = ell = 128 (a square Omega): the core is positive definite exactly
    when the shift exceeds the negative eigenvalue, which takes `retries`
    tenfold increases; the device ends at the oracle's shift and eigenvalues."""
    pr = small
    n = pr.orc.n
    Om, Y0, _, _ = _indefinite_sketch(n, 1e-3, ratio, seed=21)
    V, lam, nu = osk.nystrom_from_sketch(Om, Y0)
    nu0 = np.sqrt(n) * osk.EPS64 * np.linalg.norm(Y0, 2)
    assert nu == pytest.approx(10.0 ** retries * nu0, rel=1e-14)
    pc = pr.gpu.build_precond_from_sketch(to_dev(Om), to_dev(Y0))
    glam, gnu = pc.info()
    assert gnu == pytest.approx(nu, rel=1e-10)
    assert np.max(np.abs(np.sort(glam) - np.sort(lam))) <= 1e-8 * np.max(lam)
    R = np.random.default_rng(5).standard_normal((n, 3))
    assert relerr(to_np(pc.apply(to_dev(R))), osk.lmp_apply(V, lam, R)) <= 1e-8


def test_nystrom_shift_gives_up_with_enotspd(small):
    from paper_2401_15758_amd import rp4d
    pr = small
    Om, Y0, _, _ = _indefinite_sketch(pr.orc.n, 1e-3, 3000.0, seed=22)
    with pytest.raises(osk.NotSPDError):
        osk.nystrom_from_sketch(Om, Y0)
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.build_precond_from_sketch(to_dev(Om), to_dev(Y0))
    assert e.value.code == rp4d.ENOTSPD


def test_zero_omega_column_is_enotspd_on_both_sides(small):
    """A zero column of Omega makes the core singular at every shift."""
    from paper_2401_15758_amd import rp4d
    pr = small
    Om = inputs.omega(pr.orc.n, 10, seed=23)
    Om[:, 4] = 0.0
    with pytest.raises(osk.NotSPDError):
        ogn.build_precond(pr.orc, pr.otraj, "nystrom", Om)
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.build_precond(pr.traj, rp4d.NYSTROM, 10, omega=to_dev(Om))
    assert e.value.code == rp4d.ENOTSPD


@pytest.mark.parametrize("rtol", [1.0, 2.0])
def test_pcg_tolerance_met_by_the_zero_start(small, rtol):
    """rtol >= 1: ||r_0|| = ||b|| <= rtol ||b||, so x = 0 after no iteration,
    as in the oracle; the speculative first iteration is discarded."""
    torch = need_gpu()
    pr = small
    b = np.random.default_rng(31).standard_normal(pr.orc.n)
    xr, ir = opcg(lambda v: pr.orc.hessian(pr.otraj, v), b, rtol=rtol)
    assert ir["iters"] == 0 and not np.any(xr)
    before = pr.gpu.counters()
    x, info = pr.gpu.pcg_solve(pr.traj, to_dev(b), rtol=rtol, x=torch.full((pr.orc.n,), 7.0, dtype=torch.float64,
                                                                             device="cuda"))
    after = pr.gpu.counters()
    assert info["iters"] == 0 and info["converged"] and info["relres"] == pytest.approx(ir["relres"])
    assert torch.count_nonzero(x).item() == 0
    assert after["tlm_online"] == before["tlm_online"]


def test_nonfinite_inputs_are_reported():
    """A NaN in the observations or in the state reaches the host as
    ENONFINITE (FWD cost, GN step), never as a silent result."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    pr = Pair(inputs.CFG_SMALL, seed=3)
    y = pr.orc.y.reshape(-1).copy()
    y[7] = np.nan
    pr.gpu.set_data(to_dev(pr.orc.xb), to_dev(y))
    tr = pr.gpu.traj()
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.fwd(to_dev(pr.orc.xb), tr)
    assert e.value.code == rp4d.ENONFINITE
    st = pr.gpu.gn_state()
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.gn_step(st, sketch=rp4d.NYSTROM, ell=8, seed=1)
    assert e.value.code == rp4d.ENONFINITE
    # clean data again, NaN in the state
    pr.gpu.set_data(to_dev(pr.orc.xb), to_dev(pr.orc.y.reshape(-1)))
    x = pr.orc.xb.copy()
    x[3] = np.inf
    with pytest.raises(rp4d.Rp4dError) as e:
        pr.gpu.fwd(to_dev(x), tr)
    assert e.value.code == rp4d.ENONFINITE
    torch.cuda.synchronize()


def test_gn_step_failing_mid_sketch_leaves_the_state_usable():
    """An argument error raised inside the sketch's TLM loop (an invalid sweep
    tiling, found at its first launch, after FWD launches were enqueued on the
    side stream) leaves the GN state, its trajectory and the problem usable:
    after the tiling is restored, three steps give bitwise the iterates of a
    problem that never failed."""
    torch = need_gpu()
    from paper_2401_15758_amd import rp4d
    cfg = inputs.CFG_SMALL
    ctx = rp4d.Context(0)

    def problem():
        pr = Pair(cfg, seed=0, ctx=ctx)
        return pr.gpu

    def steps(p, st):
        for i in range(3):
            p.gn_step(st, sketch=rp4d.NYSTROM, ell=20, seed=40 + i, rtol=1e-10)
        v, x = st.get()
        torch.cuda.synchronize()
        return v.clone(), x.clone()

    ref = steps(*(lambda p: (p, p.gn_state()))(problem()))
    p = problem()
    st = p.gn_state()
    p.set_sweep_tiling(k=20, ppt=2, kc=2, threads=64, tile=10 ** 6, steps=4, mode=rp4d.MODE_TLM, xch=rp4d.XCH_WAVE)
    with pytest.raises(rp4d.Rp4dError) as e:
        p.gn_step(st, sketch=rp4d.NYSTROM, ell=20, seed=40, rtol=1e-10)
    assert e.value.code == rp4d.EINVAL
    p.set_sweep_tiling(k=20, mode=rp4d.MODE_TLM)          # back to the default tiling
    st.reset()
    got = steps(p, st)
    assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])


def test_device_philox_matches_the_oracle_stream(small):
    """The library's draws (rp4d_philox_normal) against the oracle's
    implementation of the same published generator and mapping: equal up to
    the rounding of log, cos and sin."""
    torch = need_gpu()
    pr = small
    for seed, count in ((0, 4097), (12345, 1000), ((1 << 40) + 7, 64)):
        out = torch.empty(count, dtype=torch.float64, device="cuda")
        pr.ctx.philox_normal(seed, count, out)
        ref = orng.normal(seed, count)
        assert np.max(np.abs(to_np(out) - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
