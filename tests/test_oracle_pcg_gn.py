"""Pins of the PCG and Gauss-Newton oracle: PCG against a dense direct solve of
the explicitly formed Hessian, finite termination with an exact preconditioner, the
iteration bound by the number of distinct eigenvalues, the exact GN step on a
linear model, descent of J, the reuse test value for an exact preconditioner, and
the counting identities of Tables 2 and 4."""
import numpy as np
import pytest

from oracle import burgers as bg
from oracle import gn, sketch
from oracle.pcg import pcg
from oracle.problem import Problem, burgers_problem
from paper_2401_15758_amd import inputs


def test_pcg_matches_dense_solve(small_problem, small_dense):
    p = small_problem
    traj, Hs, _ = small_dense
    b = np.random.default_rng(1).standard_normal(p.n)
    x, info = pcg(lambda v: p.hessian(traj, v), b, rtol=1e-12)
    ref = np.linalg.solve(np.eye(p.n) + Hs, b)
    kap = np.linalg.cond(np.eye(p.n) + Hs)
    assert info['converged']
    assert np.linalg.norm(x - ref) <= 10 * kap * 1e-12 * np.linalg.norm(ref)


def test_pcg_exact_preconditioner_one_iteration(small_dense):
    _, Hs, _ = small_dense
    n = Hs.shape[0]
    w, U = np.linalg.eigh(Hs)
    w = np.maximum(w, 0)
    b = np.random.default_rng(2).standard_normal(n)
    x, info = pcg(lambda v: v + Hs @ v, b, prec=lambda r: sketch.lmp_apply(U, w, r), rtol=1e-10)
    assert info['iters'] <= 2


def test_pcg_iterations_bounded_by_distinct_eigenvalues():
    rng = np.random.default_rng(3)
    n = 60
    U, _ = np.linalg.qr(rng.standard_normal((n, 4)))
    H = (U * np.array([5.0, 3.0, 2.0, 0.5])) @ U.T     # I+H has 5 distinct eigenvalues
    b = rng.standard_normal(n)
    _, info = pcg(lambda v: v + H @ v, b, rtol=1e-12)
    assert info['iters'] <= 5


class _HeatModel:
    """Linear test model (u_t = nu u_xx, RK4): the Burgers TLM around u = 0."""
    def __init__(self, n, nu, dt):
        self.n, self.nu, self.dt = n, nu, dt
        self.dx = 1.0 / n

    def _step(self, u):
        return bg.tlm_step(np.zeros(self.n), u, self.dt, self.nu, self.dx)

    def fwd(self, x0, nsteps):
        tr = [np.asarray(x0, dtype=np.float64)]
        for _ in range(nsteps):
            tr.append(self._step(tr[-1]))
        return np.array(tr)

    def tlm(self, traj, d0, obs_steps):
        return bg.tlm(np.zeros_like(traj), d0, self.dt, self.nu, self.dx, obs_steps)

    def adj(self, traj, forcings, obs_steps):
        return bg.adj(np.zeros_like(traj), forcings, self.dt, self.nu, self.dx, obs_steps)

    def obs_index(self, stride):
        return np.arange(0, self.n, stride)

    def bhalf(self, V, sigma_b, L):
        from oracle.prior import bhalf_1d
        return bhalf_1d(V, self.dx, sigma_b, L)


def test_gn_step_exact_on_linear_model():
    n = 64
    model = _HeatModel(n, 0.01, 1e-3)
    p = Problem(model=model, nsteps=20, obs_stride=4, obs_every=5, sigma_o=0.01, sigma_b=0.05, L_b=0.05)
    rng = np.random.default_rng(4)
    x_true = np.sin(2 * np.pi * np.arange(n) / n)
    p.xb = x_true + p.bhalf(rng.standard_normal(n))
    p.y = p.observe(p.fwd(x_true)) + 0.01 * rng.standard_normal((p.n_t, p.n_obs))
    v0 = np.zeros(n)
    _, g0, _, _ = p.cost_grad(v0)
    v1, dv, x1, info = gn.gn_step(p, v0, method='none', rtol=1e-13)
    _, g1, _, _ = p.cost_grad(v1)
    assert np.linalg.norm(g1) <= 1e-9 * np.linalg.norm(g0)


def test_gn_decreases_cost_and_counters(small_cfg):
    p = burgers_problem(small_cfg, inputs.draws(small_cfg, seed=0))
    v = np.zeros(p.n)
    c = dict(fwd=0, tlm_on=0, adj_on=0, tlm_off=0, adj_off=0)
    Js, iters = [], []
    for k in range(3):
        Om = inputs.omega(p.n, 20, seed=1000 + k)
        v, dv, x, info = gn.gn_step(p, v, method='nystrom', Omega=Om, rtol=1e-9, counters=c)
        Js.append(info['J'])
        iters.append(info['pcg']['iters'])
    Js.append(p.cost(v))
    assert all(b < a for a, b in zip(Js[:2], Js[1:3]))
    assert Js[-1] <= Js[-2] * (1 + 1e-12)
    assert c['tlm_on'] == sum(iters)
    assert c['adj_on'] == sum(iters) + 3
    assert c['tlm_off'] == c['adj_off'] == 20 * 3
    assert c['fwd'] == 3


def test_preconditioner_reduces_iterations(small_cfg):
    p = burgers_problem(small_cfg, inputs.draws(small_cfg, seed=0))
    v0 = np.zeros(p.n)
    _, _, _, i0 = gn.gn_step(p, v0, method='none', rtol=1e-9)
    _, _, _, i1 = gn.gn_step(p, v0, method='nystrom', Omega=inputs.omega(p.n, 20), rtol=1e-9)
    _, _, _, i2 = gn.gn_step(p, v0, method='randsvd', Omega=inputs.omega(p.n, 20), rtol=1e-9)
    assert i1['pcg']['iters'] < i0['pcg']['iters']
    assert i2['pcg']['iters'] < i0['pcg']['iters']


def test_kappa_re_exact_preconditioner_is_one(small_problem, small_dense):
    p = small_problem
    traj, Hs, _ = small_dense
    w, U = np.linalg.eigh(Hs)
    w = np.maximum(w, 0)
    k = gn.kappa_re(p, traj, U, w, inputs.unit_vector(p.n))
    assert k == pytest.approx(1.0, abs=1e-9)
    # and in general kappa_re <= ||(I + H) P||_2
    Om = inputs.omega(p.n, 5)
    V, lam, _ = sketch.nystrom(lambda X: Hs @ X, Om)
    k2 = gn.kappa_re(p, traj, V, lam, inputs.unit_vector(p.n))
    Pm = sketch.lmp_apply(V, lam, np.eye(p.n))
    assert k2 <= np.linalg.norm((np.eye(p.n) + Hs) @ Pm, 2) * (1 + 1e-10)


class _Toy:
    """cost(v) = 1/2 |v|^2 + 5 sum v^4 (quartic: a full step along -grad overshoots)."""

    @staticmethod
    def cost(v):
        return 0.5 * float(v @ v) + 5.0 * float(np.sum(v ** 4))


def test_armijo_returns_the_largest_halving_that_passes():
    from oracle import gn as ogn
    rng = np.random.default_rng(3)
    for _ in range(5):
        v = rng.standard_normal(6)
        g = v + 20.0 * v ** 3
        dv = -3.0 * g
        J0 = _Toy.cost(v)
        alpha, trials = ogn.armijo(_Toy, v, J0, g, dv)
        ok = lambda a: _Toy.cost(v + a * dv) <= J0 + 1e-4 * a * float(g @ dv)
        assert ok(alpha)
        assert alpha == 1.0 or not ok(2.0 * alpha)
        assert trials == int(round(np.log2(1.0 / alpha))) + 1


def test_line_search_on_an_inexact_sketchsolv_step():
    """SketchSolv with a 2-column sketch on the wall-bounded workload: the full
    step raises the cost 5.8-fold, half a step still raises it, a quarter step
    lowers it (margins of 28-40 % of J, so the decision is robust)."""
    from oracle import gn as ogn
    from oracle.problem import make_problem
    cfg = inputs.CFG_WALL_SMALL
    orc = make_problem(cfg, inputs.draws(cfg, seed=0))
    Om = inputs.omega(orc.n, 2, seed=1000)
    c = dict(fwd=0, tlm_on=0, adj_on=0, tlm_off=0, adj_off=0)
    v1, dv, _, info = ogn.gn_step(orc, np.zeros(orc.n), method='nystrom', Omega=Om, solve='sketch',
                                  line_search=True, counters=c)
    assert info['alpha'] == 0.25 and info['ls_trials'] == 3
    assert np.allclose(v1, 0.25 * dv)
    assert orc.cost(v1) < info['J'] and c['fwd'] == 1 + 3
