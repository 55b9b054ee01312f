"""Pins of the oracle's SketchSolv step (Sec. 3.2.1, eq. (dxsol)).

In the v-form (x = x_b + Gamma^{1/2} v) the Gamma^{-1}-norm of a step in x is
the 2-norm of the step in v, so the error theorem of Sec. 4 (error in solve)
reads |dv - dv_hat| / |dv| <= |H - H_hat|_2 with dv the exact GN step (a dense
solve of (I + H) dv = -g_v here) and dv_hat the SketchSolv step.  The bound is
checked for all three sketches on the 128-point Burgers workload; SketchPrec
(PCG) is checked against the same dense solve."""
import numpy as np
import pytest

from oracle import gn as ogn
from oracle.problem import burgers_problem
from paper_2401_15758_amd import inputs


@pytest.fixture(scope="module")
def dense():
    cfg = inputs.CFG_SMALL
    orc = burgers_problem(cfg, inputs.draws(cfg, seed=0))
    v0 = np.zeros(orc.n)
    _, g, traj, _ = orc.cost_grad(v0)
    H = orc.misfit_hessian(traj, np.eye(orc.n))
    H = 0.5 * (H + H.T)
    dv = np.linalg.solve(np.eye(orc.n) + H, -g)
    return orc, v0, H, dv


@pytest.mark.parametrize("method,ell", [("nystrom", 10), ("nystrom", 30), ("randsvd", 12), ("randsvd", 30),
                                        ("singleview", 15), ("singleview", 30)])
def test_sketchsolv_error_bound(dense, method, ell):
    orc, v0, H, dv = dense
    Om = inputs.omega(orc.n, ell, seed=300 + ell)
    arg = (Om, np.random.default_rng(ell).standard_normal((orc.m, 2 * ell + 1))) if method == "singleview" else Om
    _, dvh, _, info = ogn.gn_step(orc, v0, method=method, Omega=arg, solve='sketch')
    V, lam = info['precond']
    E = np.linalg.norm(H - (V * lam) @ V.T, 2)
    err = np.linalg.norm(dv - dvh) / np.linalg.norm(dv)
    assert info['pcg']['iters'] == 0
    assert err <= E * (1 + 1e-8) + 1e-12
    assert err > 0.0


def test_sketchprec_reaches_the_dense_step(dense):
    orc, v0, H, dv = dense
    Om = inputs.omega(orc.n, 20, seed=320)
    _, dvp, _, info = ogn.gn_step(orc, v0, method='nystrom', Omega=Om, rtol=1e-12)
    assert np.linalg.norm(dvp - dv) <= 1e-10 * np.linalg.norm(dv)


def test_sketchsolv_needs_a_sketch(dense):
    orc, v0, _, _ = dense
    with pytest.raises(ValueError):
        ogn.gn_step(orc, v0, method='none', solve='sketch')
