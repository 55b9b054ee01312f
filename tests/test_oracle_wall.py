"""Pins of the oracle's wall-bounded Burgers model (Sec. 5.1: Dirichlet walls,
central differences, RK3-TVD, discrete RK TLM / ADJ) and of the paper's prior
Gamma = (alpha I - beta Lap*)^{-2}, against facts fixed by the mathematics:
  * central differences are exact on a quadratic that vanishes at the walls;
  * the Jacobian and its transpose equal a dense matrix assembled entry by entry;
  * on a pure diffusion mode (amplitude small enough that advection is below
    roundoff) one step multiplies the mode by the RK3 stability polynomial
    1 + z + z^2/2 + z^3/6 at z = h nu eig(Lap*)/dx^2, with the Dirichlet
    eigenvalue -4 sin^2(pi/(2(n+1)));
  * the TLM is the derivative of the forward model (second-order Taylor
    remainder) and the ADJ its transpose (dot-product test);
  * the prior's sine modes are eigenvectors with eigenvalue
    1/(alpha + 4 beta sin^2(j pi/(2(n+1)))).
"""
import numpy as np
import pytest

from oracle import burgers_dirichlet as bw
from oracle import prior as opr
from oracle.problem import make_problem
from paper_2401_15758_amd import inputs


def _grid(n):
    dx = 1.0 / (n + 1)
    return (np.arange(n) + 1) * dx, dx


def test_rhs_exact_on_a_wall_quadratic():
    n, nu = 37, 0.07
    x, dx = _grid(n)
    u = x * (1.0 - x)
    assert np.allclose(bw.rhs(u, nu, dx), -u * (1.0 - 2.0 * x) - 2.0 * nu, atol=1e-12)


def test_jacobian_and_transpose_match_the_dense_matrix():
    rng = np.random.default_rng(0)
    n, nu = 17, 0.1
    _, dx = _grid(n)
    Y = rng.standard_normal(n)
    J = bw.jac_matrix_loop(Y, nu, dx)
    D = rng.standard_normal((n, 3))
    assert np.allclose(bw.jac(Y, D, nu, dx), J @ D, rtol=1e-12, atol=1e-9)
    assert np.allclose(bw.jac_t(Y, D, nu, dx), J.T @ D, rtol=1e-12, atol=1e-9)
    assert np.allclose(bw.jac(Y, D[:, 0], nu, dx), J @ D[:, 0], rtol=1e-12, atol=1e-9)


def test_one_step_on_a_diffusion_mode_is_the_rk3_polynomial():
    n, nu, h, j = 63, 0.1, 1e-3, 40
    x, dx = _grid(n)
    eps = 1e-12
    u = eps * np.sin(j * np.pi * x)
    z = h * nu * (-4.0 * np.sin(j * np.pi / (2 * (n + 1))) ** 2) / dx ** 2
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert -2.0 < z < -1.0
    assert np.allclose(bw.rk3_step(u, h, nu, dx), R * u, rtol=1e-9, atol=1e-9 * eps)


def test_tlm_is_the_derivative_and_adj_its_transpose():
    rng = np.random.default_rng(1)
    n, nu, h = 31, 0.1, 2e-4
    x, dx = _grid(n)
    u = np.sin(np.pi * x) + 0.3 * np.sin(3 * np.pi * x)
    d = rng.standard_normal(n)
    base = bw.rk3_step(u, h, nu, dx)
    lin = bw.tlm_step(u, d, h, nu, dx)
    r = [np.linalg.norm(bw.rk3_step(u + e * d, h, nu, dx) - base - e * lin) for e in (1e-3, 5e-4)]
    assert 3.5 < r[0] / r[1] < 4.5                   # second-order remainder
    L = rng.standard_normal((n, 2))
    D = rng.standard_normal((n, 2))
    lhs = np.sum(bw.tlm_step(u, D, h, nu, dx) * L)
    rhs = np.sum(D * bw.adj_step(u, L, h, nu, dx))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_window_operators_pass_the_dot_product_test():
    cfg = inputs.CFG_WALL_SMALL
    pr = make_problem(cfg, inputs.draws(cfg, seed=3))
    tr = pr.fwd(pr.xb)
    rng = np.random.default_rng(4)
    V = rng.standard_normal((pr.n, 2))
    W = rng.standard_normal((pr.n_t, pr.n_obs, 2))
    lhs = np.sum(pr.A(tr, V) * W)
    rhs = np.sum(V * pr.AT(tr, W))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    assert pr.n_obs == 16 and pr.n_t == 10 and list(pr.obs_idx[:2]) == [5, 11]


@pytest.mark.parametrize("j", [1, 2, 17, 40])
def test_prior_sine_modes_are_eigenvectors(j):
    n, a, b = 49, 0.5, 500.0
    x, _ = _grid(n)
    s = np.sin(j * np.pi * x)
    lam = 1.0 / (a + 4.0 * b * np.sin(j * np.pi / (2 * (n + 1))) ** 2)
    assert np.allclose(opr.bhalf_spde_1d(s, a, b), lam * s, rtol=1e-12, atol=1e-15)


def test_paper_configuration_shape():
    cfg = inputs.CFG_WALL
    assert inputs.n_obs(cfg) == 15 and inputs.n_t(cfg) == 20
    assert 4.0 * cfg['nu'] * cfg['dt'] * (cfg['n'] + 1) ** 2 <= inputs.RK3_DIFFUSIVE_LIMIT
    x = inputs.truth(cfg)
    assert abs(x[199] - 1.0) < 1e-15                 # sin(pi/2) at the mid node
