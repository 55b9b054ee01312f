"""Oracle: the SC-4DVAR problem in control-variable form.

Test infrastructure only (see ``oracle/__init__``).

Definitions followed:
  * model x_i = M_{t0->ti}(x_0)                      Sec. 2.1, eq. (model)
  * observations y_i = O(x_true_i) + eps_i, eps ~ N(0, R_i), R_i = sigma_o^2 I
                                                      Sec. 2.1
  * cost J (4dvar_cf), gradient (4dvar_gradient), GN Hessian (4dvar_hessian)
  * prior-preconditioned factorisation H = Gamma^{-1/2}(I + A^T A)Gamma^{-1/2},
    A = [R_i^{-1/2} O_i M_i Gamma^{1/2}]_i, m = n_obs n_t      eq. (Rhalf)

Control-variable reading: the iterate is tracked as v = Gamma^{-1/2}(x - x_b),
x = x_b + Gamma^{1/2} v, v^(0) = 0 (the paper starts at x^(0) = x_b).  Then
J(v) = 1/2 |v|^2 + 1/2 sum_i |R^{-1/2}(O x_{s_i} - y_i)|^2, its gradient is
g_v = v + A^T d with d_i = R^{-1/2}(O x_{s_i} - y_i), and its GN Hessian is I + A^T A.
This is Gamma^{1/2} times the paper's gradient and the same linear system as
eq. (gniterf1) / (pcgsystem); it never forms Gamma^{-1/2}, which does not exist
numerically for the Gaussian-kernel prior.

Observation operator: linear selection of every ``obs_stride``-th grid point
(2-D: every stride-th cell in both directions, flattened j*nx+i in increasing
order) at steps s_i = i*obs_every, i = 1..floor(N/obs_every) (t = 0 is not
observed, y_i exists for 1 <= i <= n_t).  Observation-space arrays are shaped
(n_t, n_obs[, k]).
"""
from dataclasses import dataclass, field
import numpy as np

from . import burgers as _burgers
from . import burgers_dirichlet as _bwall
from . import bve as _bve
from . import prior as _prior


@dataclass
class BurgersModel:
    """Periodic Burgers + RK4 (see ``oracle.burgers``)."""
    n: int
    nu: float
    dt: float

    @property
    def dx(self):
        return 1.0 / self.n

    def fwd(self, x0, nsteps):
        return _burgers.fwd(np.asarray(x0, dtype=np.float64), self.dt, nsteps, self.nu, self.dx)

    def tlm(self, traj, d0, obs_steps):
        return _burgers.tlm(traj, d0, self.dt, self.nu, self.dx, obs_steps)

    def adj(self, traj, forcings, obs_steps):
        return _burgers.adj(traj, forcings, self.dt, self.nu, self.dx, obs_steps)

    def obs_index(self, stride):
        return np.arange(0, self.n, stride)

    def bhalf(self, V, sigma_b, L):
        return _prior.bhalf_1d(V, self.dx, sigma_b, L)


@dataclass
class WallBurgersModel:
    """The paper's Burgers setup: Dirichlet walls, RK3-TVD, the SPDE prior
    (see ``oracle.burgers_dirichlet``, ``oracle.prior.bhalf_spde_1d``).
    Observations at nodes stride-1, 2 stride-1, ... (x = stride dx, 2 stride dx, ...)."""
    n: int
    nu: float
    dt: float
    alpha: float
    beta: float

    @property
    def dx(self):
        return 1.0 / (self.n + 1)

    def fwd(self, x0, nsteps):
        return _bwall.fwd(np.asarray(x0, dtype=np.float64), self.dt, nsteps, self.nu, self.dx)

    def tlm(self, traj, d0, obs_steps):
        return _bwall.tlm(traj, d0, self.dt, self.nu, self.dx, obs_steps)

    def adj(self, traj, forcings, obs_steps):
        return _bwall.adj(traj, forcings, self.dt, self.nu, self.dx, obs_steps)

    def obs_index(self, stride):
        return np.arange(stride - 1, self.n, stride)

    def bhalf(self, V, sigma_b, L):
        return _prior.bhalf_spde_1d(V, self.alpha, self.beta)


@dataclass
class Problem:
    """One SC-4DVAR problem: model, window, observation layout, prior, data."""
    model: object
    nsteps: int
    obs_stride: int
    obs_every: int
    sigma_o: float
    sigma_b: float
    L_b: float
    xb: np.ndarray = None
    y: np.ndarray = None          # (n_t, n_obs)
    obs_idx: np.ndarray = field(init=False)
    obs_steps: np.ndarray = field(init=False)

    def __post_init__(self):
        self.obs_idx = self.model.obs_index(self.obs_stride)
        nt = self.nsteps // self.obs_every
        self.obs_steps = self.obs_every * np.arange(1, nt + 1)

    @property
    def n(self):
        return self.model.n

    @property
    def n_obs(self):
        return len(self.obs_idx)

    @property
    def n_t(self):
        return len(self.obs_steps)

    @property
    def m(self):
        return self.n_obs * self.n_t

    # -- building blocks ----------------------------------------------------
    def bhalf(self, V):
        return self.model.bhalf(np.asarray(V, dtype=np.float64), self.sigma_b, self.L_b)

    def fwd(self, x0):
        return self.model.fwd(x0, self.nsteps)

    def observe(self, traj):
        """O x_{s_i} for every observation step: (n_t, n_obs)."""
        return np.stack([traj[s][self.obs_idx] for s in self.obs_steps])

    def A(self, traj, V):
        """A V = [R^{-1/2} O M_i Gamma^{1/2} V]_i  -> (n_t, n_obs[, k])."""
        d0 = self.bhalf(V)
        states = self.model.tlm(traj, d0, self.obs_steps)
        return np.stack([st[self.obs_idx] / self.sigma_o for st in states])

    def AT(self, traj, W):
        """A^T W = Gamma^{1/2} sum_i M_i^T O^T R^{-1/2} W_i; W is (n_t, n_obs[, k])."""
        W = np.asarray(W, dtype=np.float64)
        shape = (self.n,) + W.shape[2:]
        forcings = []
        for i in range(self.n_t):
            f = np.zeros(shape)
            f[self.obs_idx] = W[i] / self.sigma_o
            forcings.append(f)
        lam0 = self.model.adj(traj, forcings, self.obs_steps)
        return self.bhalf(lam0)

    def misfit_hessian(self, traj, V):
        """H V = A^T A V (data-misfit part, eq. (Rhalf))."""
        return self.AT(traj, self.A(traj, V))

    def hessian(self, traj, V):
        """(I + H) V: the prior-preconditioned GN Hessian (eq. (pcgsystem))."""
        V = np.asarray(V, dtype=np.float64)
        return V + self.misfit_hessian(traj, V)

    # -- cost and gradient ---------------------------------------------------
    def state(self, v):
        return self.xb + self.bhalf(v)

    def innovations(self, traj):
        """d_i = R^{-1/2}(O x_{s_i} - y_i): (n_t, n_obs)."""
        return (self.observe(traj) - self.y) / self.sigma_o

    def cost_grad(self, v):
        """J(v), g_v = v + A^T d and the trajectory at x = x_b + Gamma^{1/2} v
        (eqs. (4dvar_cf), (4dvar_gradient) in control-variable form)."""
        v = np.asarray(v, dtype=np.float64)
        x = self.state(v)
        traj = self.fwd(x)
        d = self.innovations(traj)
        J = 0.5 * float(v @ v) + 0.5 * float(np.sum(d * d))
        g = v + self.AT(traj, d)
        return J, g, traj, x

    def cost(self, v):
        x = self.state(v)
        traj = self.fwd(x)
        d = self.innovations(traj)
        return 0.5 * float(v @ v) + 0.5 * float(np.sum(d * d))


def synthesize(prob, x_true, xi, eta):
    """Synthetic data (Sec. 5.1 'Data and Background'): x_b = x_true + Gamma^{1/2} xi,
    y_i = O x_true(s_i) + sigma_o eta_i with the truth propagated by the same model
    (perfect-model assumption, Sec. 2.1).  Returns (x_b, y)."""
    xb = np.asarray(x_true, dtype=np.float64) + prob.bhalf(xi)
    traj = prob.fwd(x_true)
    y = prob.observe(traj) + prob.sigma_o * np.asarray(eta, dtype=np.float64).reshape(prob.n_t, prob.n_obs)
    return xb, y


def burgers_problem(cfg, draws=None):
    """Build a Burgers Problem from a plain config dict (keys: n, nu, dt, nsteps,
    obs_stride, obs_every, sigma_o, sigma_b, L_b) and, optionally, raw draws
    (dict with x_true, xi, eta) from which the data are synthesised."""
    model = BurgersModel(n=int(cfg['n']), nu=float(cfg['nu']), dt=float(cfg['dt']))
    prob = Problem(model=model, nsteps=int(cfg['nsteps']), obs_stride=int(cfg['obs_stride']),
                   obs_every=int(cfg['obs_every']), sigma_o=float(cfg['sigma_o']),
                   sigma_b=float(cfg['sigma_b']), L_b=float(cfg['L_b']))
    if draws is not None:
        prob.xb, prob.y = synthesize(prob, draws['x_true'], draws['xi'], draws['eta'])
    return prob


def bve_problem(cfg, draws=None):
    """Build a barotropic-vorticity Problem from a config dict (keys: nx, ny, nu, dt,
    nsteps, obs_stride, obs_every, sigma_o, sigma_b, L_b in cells) and optional draws."""
    model = _bve.BVEModel(nx=int(cfg['nx']), ny=int(cfg['ny']), nu=float(cfg['nu']), dt=float(cfg['dt']))
    prob = Problem(model=model, nsteps=int(cfg['nsteps']), obs_stride=int(cfg['obs_stride']),
                   obs_every=int(cfg['obs_every']), sigma_o=float(cfg['sigma_o']),
                   sigma_b=float(cfg['sigma_b']), L_b=float(cfg['L_b']))
    if draws is not None:
        prob.xb, prob.y = synthesize(prob, draws['x_true'], draws['xi'], draws['eta'])
    return prob


def wall_burgers_problem(cfg, draws=None):
    """The paper's Burgers setup from a config dict (keys: n, nu, dt, nsteps,
    obs_stride, obs_every, sigma_o, prior_alpha, prior_beta) and optional draws."""
    model = WallBurgersModel(n=int(cfg['n']), nu=float(cfg['nu']), dt=float(cfg['dt']),
                             alpha=float(cfg['prior_alpha']), beta=float(cfg['prior_beta']))
    prob = Problem(model=model, nsteps=int(cfg['nsteps']), obs_stride=int(cfg['obs_stride']),
                   obs_every=int(cfg['obs_every']), sigma_o=float(cfg['sigma_o']), sigma_b=0.0, L_b=0.0)
    if draws is not None:
        prob.xb, prob.y = synthesize(prob, draws['x_true'], draws['xi'], draws['eta'])
    return prob


def make_problem(cfg, draws=None):
    kind = cfg.get('model')
    if kind == 'bve':
        return bve_problem(cfg, draws)
    if kind == 'burgers_wall':
        return wall_burgers_problem(cfg, draws)
    return burgers_problem(cfg, draws)
