"""Pins of the barotropic-vorticity oracle: Arakawa's conservation identities and
antisymmetry, convergence of J_A to the continuous Jacobian, the spectral inverse
Laplacian on exact Fourier modes, the adjoint against an explicitly transposed
Jacobian matrix, the TLM against complex-step derivatives, the RK4 dot-product
test, and the closed-form diffusion mode around a state at rest."""
import numpy as np
import pytest

from oracle import bve
from oracle.problem import bve_problem
from paper_2401_15758_amd import inputs


def _f(ny, nx, seed, k=None):
    r = np.random.default_rng(seed)
    return r.standard_normal((ny, nx) if k is None else (ny, nx, k))


def test_arakawa_conservation_and_antisymmetry():
    a, b = _f(16, 16, 1), _f(16, 16, 2)
    d = 1.0 / 16
    J = bve.arakawa(a, b, d)
    scale = np.abs(J).max()
    assert abs(J.sum()) <= 1e-12 * scale * J.size
    assert abs(np.sum(a * J)) <= 1e-12 * scale * np.abs(a).sum()
    assert abs(np.sum(b * J)) <= 1e-12 * scale * np.abs(b).sum()
    assert np.allclose(bve.arakawa(b, a, d), -J, atol=1e-12 * scale)


def test_arakawa_trilinear_form_is_cyclic():
    a, b, c = _f(12, 12, 3), _f(12, 12, 4), _f(12, 12, 5)
    d = 1.0 / 12
    t1 = np.sum(c * bve.arakawa(a, b, d))
    t2 = np.sum(a * bve.arakawa(b, c, d))
    t3 = np.sum(b * bve.arakawa(c, a, d))
    assert t1 == pytest.approx(t2, rel=1e-12) and t1 == pytest.approx(t3, rel=1e-12)


def test_arakawa_second_order_convergence():
    errs = []
    for n in (16, 32, 64):
        x = np.arange(n) / n
        X, Y = np.meshgrid(x, x)                 # rows j = y, cols i = x
        a = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        b = np.sin(4 * np.pi * Y) + np.cos(2 * np.pi * X)
        ax = 2 * np.pi * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y)
        ay = -2 * np.pi * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
        bx = -2 * np.pi * np.sin(2 * np.pi * X)
        by = 4 * np.pi * np.cos(4 * np.pi * Y)
        ref = ax * by - ay * bx
        errs.append(np.abs(bve.arakawa(a, b, 1.0 / n) - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9), rates


def test_inverse_laplacian_on_fourier_modes():
    n = 32
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    for kx, ky in [(1, 0), (3, 2), (5, 7)]:
        z = np.cos(2 * np.pi * (kx * X + ky * Y)) + 0.3
        ref = -np.cos(2 * np.pi * (kx * X + ky * Y)) / ((2 * np.pi) ** 2 * (kx ** 2 + ky ** 2))
        assert np.allclose(bve.inv_lap(z), ref, atol=1e-15)


def test_adjoint_is_explicit_transpose_of_jacobian():
    n = 6
    d, nu = 1.0 / n, 0.01
    Y = _f(n, n, 6)
    cols = []
    for e in np.eye(n * n):
        cols.append(bve.jac(Y, e.reshape(n, n), nu, d).reshape(-1))
    Jm = np.array(cols).T
    for e_idx in (0, 7, 20):
        lam = np.eye(n * n)[e_idx].reshape(n, n)
        assert np.allclose(bve.jac_t(Y, lam, nu, d).reshape(-1), Jm[e_idx, :], atol=1e-10 * np.abs(Jm).max())
    L = _f(n, n, 7)
    JtL = bve.jac_t(Y, L, nu, d).reshape(-1)
    assert np.allclose(JtL, Jm.T @ L.reshape(-1), rtol=1e-12, atol=1e-10 * np.abs(Jm).max())


def test_tlm_equals_complex_step_of_fwd():
    m = bve.BVEModel(16, 16, 1e-3, 2e-3)
    x = _f(16, 16, 8).reshape(-1)
    v = _f(16, 16, 9).reshape(-1)
    eps = 1e-30
    trc = m.fwd(x + 1j * eps * v, 6)
    tr = m.fwd(x, 6)
    got = m.tlm(tr, v, [3, 6])
    for s, g in zip([3, 6], got):
        ref = np.imag(trc[s]) / eps
        assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref)


def test_rk4_dot_product():
    m = bve.BVEModel(16, 16, 1e-3, 2e-3)
    x = _f(16, 16, 10).reshape(-1)
    tr = m.fwd(x, 8)
    V = np.random.default_rng(11).standard_normal((256, 3))
    W = [np.random.default_rng(12 + i).standard_normal((256, 3)) for i in range(2)]
    TV = m.tlm(tr, V, [4, 8])
    lhs = sum(np.sum(a * b) for a, b in zip(TV, W))
    rhs = np.sum(V * m.adj(tr, W, [4, 8]))
    assert abs(lhs - rhs) <= 1e-12 * np.sqrt(sum(np.sum(a * a) for a in TV) * sum(np.sum(w * w) for w in W))


def test_diffusion_mode_closed_form_around_rest():
    n, nu, h, steps = 16, 1e-2, 1e-3, 5
    m = bve.BVEModel(n, n, nu, h)
    tr = np.zeros((steps + 1, n * n))
    x = np.arange(n) / n
    X, Y = np.meshgrid(x, x)
    d = 1.0 / n
    for kx, ky in [(1, 2), (4, 3)]:
        e = np.cos(2 * np.pi * (kx * X + ky * Y))
        mu = nu * (2 * np.cos(2 * np.pi * kx * d) + 2 * np.cos(2 * np.pi * ky * d) - 4) / d ** 2
        z = h * mu
        R = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
        got = m.tlm(tr, e.reshape(-1), [steps])[0]
        assert np.allclose(got, R ** steps * e.reshape(-1), atol=1e-13)


def test_bve_problem_operators_small_grid():
    cfg = inputs.bve_config(32, nsteps=12, obs_stride=8, obs_every=4, L_cells=3.0, ell=10)
    p = bve_problem(cfg, inputs.draws(cfg, seed=1))
    assert p.n_obs == 16 and p.n_t == 3
    tr = p.fwd(p.xb)
    V = np.random.default_rng(2).standard_normal((p.n, 2))
    W = np.random.default_rng(3).standard_normal((p.n_t, p.n_obs, 2))
    AV = p.A(tr, V)
    assert abs(np.sum(AV * W) - np.sum(V * p.AT(tr, W))) <= 1e-12 * np.linalg.norm(AV) * np.linalg.norm(W)
    # truth spectrum: unit rms, zero mean
    x = inputs.bve_truth(cfg, np.random.default_rng(0))
    assert np.sqrt(np.mean(x * x)) == pytest.approx(1.0) and abs(x.mean()) < 1e-12
