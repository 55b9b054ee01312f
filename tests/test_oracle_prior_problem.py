"""Pins of the prior square root and of the SC-4DVAR operators: S S = B against
the dense covariance, S against an eigh-based sqrtm, A^T as the transpose of A,
the gradient against finite differences of the cost, Hessian symmetry and
positivity, and the rank bound rank(H) <= m."""
import numpy as np
import pytest

from oracle import prior
from oracle.problem import burgers_problem
from paper_2401_15758_amd import inputs


@pytest.mark.parametrize("n", [128, 256])
def test_sqrt_squares_to_covariance(n):
    dx = 1.0 / n
    S = prior.sqrt_matrix_1d(n, dx, 0.05, 0.05)
    B = prior.cov_matrix_1d(n, dx, 0.05, 0.05)
    assert np.array_equal(S, S.T)
    assert np.linalg.norm(S @ S - B) <= 1e-14 * np.linalg.norm(B)


def test_sqrt_matches_eigh_sqrtm_to_conditioning():
    n = 128
    dx = 1.0 / n
    B = prior.cov_matrix_1d(n, dx, 0.05, 0.05)
    w, U = np.linalg.eigh(B)
    Sref = (U * np.sqrt(np.maximum(w, 0))) @ U.T
    S = prior.sqrt_matrix_1d(n, dx, 0.05, 0.05)
    # the eigh root is accurate only to sqrt(eps * |B|): tiny eigenvalues flip sign
    assert np.linalg.norm(S - Sref) <= 1e-6 * np.linalg.norm(S)
    # S is PSD: circulant eigenvalues are the DFT of the (positive) Gaussian kernel
    assert np.min(np.linalg.eigvalsh(S)) >= -1e-14 * np.max(np.abs(S))


def test_bhalf_2d_squares_to_separable_covariance():
    nx = ny = 64
    L = 4.0
    rng = np.random.default_rng(3)
    F = rng.standard_normal((nx * ny, 2))
    twice = prior.bhalf_2d(prior.bhalf_2d(F, nx, ny, 0.05, L), nx, ny, 0.05, L)
    B = prior.cov_matrix_2d(nx, ny, 0.05, L)
    ref = B @ F
    assert np.linalg.norm(twice - ref) <= 1e-13 * np.linalg.norm(ref)


def test_adjoint_operator_is_transpose(small_problem):
    p = small_problem
    traj = p.fwd(p.xb)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((p.n, 3))
    W = rng.standard_normal((p.n_t, p.n_obs, 3))
    AV = p.A(traj, V)
    ATW = p.AT(traj, W)
    lhs, rhs = np.sum(AV * W), np.sum(V * ATW)
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(AV) * np.linalg.norm(W)


def test_gradient_matches_central_differences(small_problem):
    p = small_problem
    rng = np.random.default_rng(6)
    v = 0.3 * rng.standard_normal(p.n)
    _, g, _, _ = p.cost_grad(v)
    for seed in range(3):
        e = np.random.default_rng(100 + seed).standard_normal(p.n)
        h = 1e-5
        fd = (p.cost(v + h * e) - p.cost(v - h * e)) / (2 * h)
        assert abs(fd - g @ e) <= 1e-7 * max(1.0, abs(g @ e))


def test_dense_hessian_symmetric_psd_and_rank(small_problem, small_dense):
    p = small_problem
    _, Hs, Hd = small_dense
    assert np.linalg.norm(Hd - Hd.T) <= 1e-12 * np.linalg.norm(Hd)
    w = np.linalg.eigvalsh(Hs)
    assert w[0] >= -1e-12 * w[-1]
    assert np.linalg.matrix_rank(Hs, tol=1e-10 * w[-1]) <= min(p.m, p.n)


def test_observation_layout(small_cfg):
    p = burgers_problem(small_cfg)
    assert list(p.obs_steps) == [10, 20, 30, 40, 50]
    assert list(p.obs_idx[:3]) == [0, 4, 8] and p.n_obs == 32 and p.m == 160


def test_synthesis_uses_truth_and_noise(small_cfg):
    d = inputs.draws(small_cfg, seed=0)
    p = burgers_problem(small_cfg, d)
    traj = p.fwd(d['x_true'])
    resid = (p.y - p.observe(traj)) / p.sigma_o
    assert np.allclose(resid, d['eta'], atol=1e-10)
    assert np.allclose(p.xb - d['x_true'], p.bhalf(d['xi']), atol=1e-15)


def test_stable_dt_reading():
    assert inputs.CFG_SMALL['dt'] == 1e-3
    dx = 1.0 / 4096
    assert inputs.CFG_LARGE['dt'] == pytest.approx(0.5 * dx * dx / 0.01)
    assert 4 * 0.01 * inputs.CFG_LARGE['dt'] / dx ** 2 <= 2.785
