"""Pins of the Burgers oracle (model, discrete RK4 TLM and ADJ) against facts that
do not come from the oracle's own formulas: a loop-assembled Jacobian, complex-step
derivatives of the nonlinear model, finite differences, the closed-form RK4
amplification factor of linear advection-diffusion, and conservation laws."""
import numpy as np
import pytest

from oracle import burgers as bg

NU, N = 0.01, 16
DX = 1.0 / N


def _rand(n, seed, k=None):
    r = np.random.default_rng(seed)
    return r.standard_normal(n if k is None else (n, k))


def test_rhs_and_jac_match_scalar_loops():
    u, d = _rand(N, 1), _rand(N, 2)
    assert np.allclose(bg.rhs(u, NU, DX), bg.rhs_loop(u, NU, DX), rtol=1e-14, atol=1e-12)
    assert np.allclose(bg.jac(u, d, NU, DX), bg.jac_loop(u, d, NU, DX), rtol=1e-14, atol=1e-12)


def test_jacobian_and_transpose_against_assembled_matrix():
    Y, d = _rand(N, 3), _rand(N, 4, k=3)
    J = bg.jac_matrix_loop(Y, NU, DX)
    assert np.allclose(bg.jac(Y, d, NU, DX), J @ d, rtol=1e-13, atol=1e-10)
    assert np.allclose(bg.jac_t(Y, d, NU, DX), J.T @ d, rtol=1e-13, atol=1e-10)


def test_jacobian_is_complex_step_derivative_of_rhs():
    u, d = _rand(N, 5), _rand(N, 6)
    h = 1e-30
    cs = np.imag(bg.rhs(u + 1j * h * d, NU, DX)) / h
    assert np.allclose(cs, bg.jac(u, d, NU, DX), rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("n,steps", [(32, 20), (128, 50)])
def test_tlm_equals_complex_step_of_fwd(n, steps):
    dx, h = 1.0 / n, 1e-3 if n == 128 else 2e-3
    x = np.sin(2 * np.pi * np.arange(n) / n) + 0.3 * _rand(n, 7)
    v = _rand(n, 8)
    eps = 1e-30
    traj_c = bg.fwd(x + 1j * eps * v, h, steps, NU, dx)
    traj = bg.fwd(x, h, steps, NU, dx)
    obs = [steps // 2, steps]
    got = bg.tlm(traj, v, h, NU, dx, obs)
    for s, g in zip(obs, got):
        ref = np.imag(traj_c[s]) / eps
        assert np.linalg.norm(g - ref) <= 1e-13 * np.linalg.norm(ref)


def test_tlm_finite_difference_second_order():
    n, h, steps = 64, 2e-3, 30
    dx = 1.0 / n
    x = np.sin(2 * np.pi * np.arange(n) / n)
    v = _rand(n, 9)
    traj = bg.fwd(x, h, steps, NU, dx)
    t = bg.tlm(traj, v, h, NU, dx, [steps])[0]
    errs = []
    for e in [1e-2, 5e-3, 2.5e-3]:
        fd = (bg.fwd(x + e * v, h, steps, NU, dx)[-1] - bg.fwd(x - e * v, h, steps, NU, dx)[-1]) / (2 * e)
        errs.append(np.linalg.norm(fd - t) / np.linalg.norm(t))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8) and np.all(rates < 2.2), (errs, rates)


@pytest.mark.parametrize("k", [1, 4])
def test_adjoint_dot_product(k):
    n, h, steps = 128, 1e-3, 50
    dx = 1.0 / n
    x = np.sin(2 * np.pi * np.arange(n) / n) + 0.5 * np.sin(4 * np.pi * np.arange(n) / n)
    traj = bg.fwd(x, h, steps, NU, dx)
    obs = [10, 20, 30, 40, 50]
    v = _rand(n, 10, k=k)
    ws = [_rand(n, 20 + i, k=k) for i in range(len(obs))]
    tv = bg.tlm(traj, v, h, NU, dx, obs)
    lhs = sum(np.sum(a * b) for a, b in zip(tv, ws))
    rhs = np.sum(v * bg.adj(traj, ws, h, NU, dx, obs))
    scale = np.sqrt(sum(np.sum(a * a) for a in tv) * sum(np.sum(w * w) for w in ws))
    assert abs(lhs - rhs) <= 1e-12 * scale


def _rk4_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


@pytest.mark.parametrize("c", [0.0, 0.7])
def test_tlm_closed_form_fourier_mode(c):
    """Around u = c the TLM is linear advection-diffusion: mode kappa is multiplied
    per step by R(h mu_kappa), mu = -i c sin(2 pi kappa/n)/dx - 4 nu/dx^2 sin^2(pi kappa/n)."""
    n, h, steps = 64, 1e-3, 7
    dx = 1.0 / n
    traj = np.full((steps + 1, n), c)
    j = np.arange(n)
    for kap in [1, 5, 17, 31]:
        e = np.exp(2j * np.pi * kap * j / n)
        mu = -1j * c * np.sin(2 * np.pi * kap / n) / dx - 4 * NU / dx ** 2 * np.sin(np.pi * kap / n) ** 2
        ref = _rk4_poly(h * mu) ** steps * e
        re = bg.tlm(traj, e.real.copy(), h, NU, dx, [steps])[0]
        im = bg.tlm(traj, e.imag.copy(), h, NU, dx, [steps])[0]
        assert np.allclose(re + 1j * im, ref, rtol=0, atol=1e-13)
        if c == 0.0:
            adj = bg.adj(traj, [e.real.copy()], h, NU, dx, [steps])
            assert np.allclose(adj, ref.real, atol=1e-13)


def test_fwd_conserves_mean_and_constant_is_fixed_point():
    n, h = 128, 1e-3
    dx = 1.0 / n
    x = np.sin(2 * np.pi * np.arange(n) / n) + 0.2 + 0.1 * _rand(n, 11)
    tr = bg.fwd(x, h, 50, NU, dx)
    assert abs(tr[-1].sum() - x.sum()) <= 1e-12 * np.abs(x).sum()
    c = np.full(n, 0.37)
    assert np.array_equal(bg.fwd(c, h, 10, NU, dx)[-1], c)


def test_rk4_step_matches_stage_states():
    n, h = 32, 1e-3
    dx = 1.0 / n
    u = _rand(n, 12)
    Y = bg.rk4_stages(u, h, NU, dx)
    K = [bg.rhs(y, NU, dx) for y in Y]
    ref = u + h * (K[0] + 2 * K[1] + 2 * K[2] + K[3]) / 6
    assert np.allclose(bg.rk4_step(u, h, NU, dx), ref, rtol=1e-15, atol=1e-15)
