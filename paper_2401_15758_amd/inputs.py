"""Seeded synthetic workloads: configurations and raw random draws.

This module holds no arithmetic of the method: it only states the workload
shapes and parameters and draws the random numbers that the method consumes
(background noise xi, observation noise eta, Gaussian test matrices Omega,
unit test vectors).  Both the HIP library (through its Python binding) and the
CPU oracle take these arrays as inputs; neither computes them.

Workloads (all synthetic; the paper's own data -- figure-only observation
locations, a spun-up gyre truth -- are not available and not needed):

  burgers-128    periodic Burgers n=128, nu=0.01, dt=1e-3, 50 RK4 steps, observe
                 every 4th point every 10 steps, sigma_o=0.01, Gaussian prior
                 sigma_b=0.05, L=0.05; sketch l=20.
  burgers-4096   same at n=4096, 500 steps, every 16th point every 25 steps,
                 sketch l=64, 3 GN iterations.  The configured dt=2.5e-5 is outside
                 RK4's stability interval at this resolution (4 nu dt/dx^2 = 16.8 >
                 2.785); the step is reduced to dt = 0.5 dx^2/nu (the step count
                 and observation cadence are kept).
  batch-64       64 independent Burgers problems, n log-uniform in [256, 4096],
                 N uniform in [50, 500], per-problem seeds; sketch l=32.
  bve-256        periodic barotropic vorticity on a 256 x 256 grid of [0,1)^2,
                 nu = 1e-4, dt = 2e-3, 200 RK4 steps, observe every 16th cell in
                 both directions every 20 steps (n_obs = 256, n_t = 10), sigma_o =
                 0.01, separable Gaussian prior sigma_b = 0.05, L = 8 cells; sketch
                 l = 100.  Truth: random-phase vorticity with |zeta_hat(k)| ~ 1/|k|
                 (energy spectrum k^-3) for 1 <= |k| <= n/3, scaled to unit rms.

  burgers-wall-399  the paper's Burgers setup (Sec. 5.1, Table 3): Dirichlet walls,
                 n = 399 interior nodes (dx = 0.0025), nu = 0.1, RK3-TVD with
                 dt = 2.5e-5, 20 observation times 0.01 apart (400 steps apart,
                 8000 steps), 15 observed nodes (every 25th from node 24: the
                 paper's locations are only drawn in a figure), R = 0.01 I,
                 prior Gamma = (0.5 I - 500 Lap*)^{-2}; truth sin(pi x); l = 15.
  burgers-wall-99   the same setup on 99 nodes, 400 steps, observations every 40
                 steps at every 6th node (parity size).

Truth: u0(x) = sin(2 pi x) + 0.5 sin(4 pi x) on x_j = j/n (periodic models);
sin(pi x) on x_j = (j + 1)/(n + 1) (wall model).
"""
import math
import numpy as np

RK4_DIFFUSIVE_LIMIT = 2.785   # RK4 real-axis stability interval (|z| <= 2.785)


def stable_dt(n, nu, dt_cfg):
    """Reading for configured steps outside RK4's stability interval: keep the
    configured step when 4 nu dt/dx^2 <= 2.785, else use dt = 0.5 dx^2 / nu."""
    dx = 1.0 / n
    if 4.0 * nu * dt_cfg / (dx * dx) <= RK4_DIFFUSIVE_LIMIT:
        return dt_cfg
    return 0.5 * dx * dx / nu


def burgers_config(n, nsteps, obs_stride, obs_every, dt_cfg=1e-3, nu=0.01,
                   sigma_o=0.01, sigma_b=0.05, L_b=0.05, ell=20, name=None):
    return dict(model='burgers', name=name or f'burgers-{n}', n=int(n), nu=float(nu),
                dt=float(stable_dt(n, nu, dt_cfg)), dt_cfg=float(dt_cfg), nsteps=int(nsteps),
                obs_stride=int(obs_stride), obs_every=int(obs_every), sigma_o=float(sigma_o),
                sigma_b=float(sigma_b), L_b=float(L_b), ell=int(ell))


CFG_SMALL = burgers_config(128, 50, 4, 10, dt_cfg=1e-3, ell=20, name='burgers-128')
CFG_LARGE = burgers_config(4096, 500, 16, 25, dt_cfg=2.5e-5, ell=64, name='burgers-4096')


def bve_config(nx, nsteps=200, obs_stride=16, obs_every=20, dt=2e-3, nu=1e-4, sigma_o=0.01, sigma_b=0.05,
               L_cells=8.0, ell=100, name=None):
    return dict(model='bve', name=name or f'bve-{nx}', nx=int(nx), ny=int(nx), n=int(nx) * int(nx), nu=float(nu),
                dt=float(dt), nsteps=int(nsteps), obs_stride=int(obs_stride), obs_every=int(obs_every),
                sigma_o=float(sigma_o), sigma_b=float(sigma_b), L_b=float(L_cells), ell=int(ell))


CFG_BVE = bve_config(256, name='bve-256')

RK3_DIFFUSIVE_LIMIT = 2.51    # RK3-TVD real-axis stability interval (|z| <= 2.51)


def wall_config(n, nsteps, obs_stride, obs_every, dt=2.5e-5, nu=0.1, sigma_o=0.1, prior_alpha=0.5,
                prior_beta=500.0, ell=15, name=None):
    return dict(model='burgers_wall', name=name or f'burgers-wall-{n}', n=int(n), nu=float(nu), dt=float(dt),
                nsteps=int(nsteps), obs_stride=int(obs_stride), obs_every=int(obs_every), sigma_o=float(sigma_o),
                prior_alpha=float(prior_alpha), prior_beta=float(prior_beta), sigma_b=0.0, L_b=0.0, ell=int(ell))


CFG_WALL = wall_config(399, 8000, 25, 400, name='burgers-wall-399')
CFG_WALL_SMALL = wall_config(99, 400, 6, 40, dt=2.5e-4, ell=12, name='burgers-wall-99')


def n_obs(cfg):
    if cfg.get('model') == 'bve':
        return len(range(0, cfg['nx'], cfg['obs_stride'])) * len(range(0, cfg['ny'], cfg['obs_stride']))
    if cfg.get('model') == 'burgers_wall':
        return len(range(cfg['obs_stride'] - 1, cfg['n'], cfg['obs_stride']))
    return len(range(0, cfg['n'], cfg['obs_stride']))


def n_t(cfg):
    return cfg['nsteps'] // cfg['obs_every']


def truth(cfg):
    if cfg.get('model') == 'burgers_wall':
        return np.sin(np.pi * (np.arange(cfg['n']) + 1) / (cfg['n'] + 1))
    x = np.arange(cfg['n']) / cfg['n']
    return np.sin(2 * np.pi * x) + 0.5 * np.sin(4 * np.pi * x)


def bve_truth(cfg, rng):
    """Random-phase vorticity with |zeta_hat(k)| ~ 1/|k| on 1 <= |k| <= nx/3, unit rms,
    flattened j*nx + i."""
    nx, ny = cfg['nx'], cfg['ny']
    kx = np.fft.rfftfreq(nx, 1.0 / nx)
    ky = np.fft.fftfreq(ny, 1.0 / ny)
    kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    amp = np.where((kk >= 1) & (kk <= nx / 3), 1.0 / np.maximum(kk, 1.0), 0.0)
    phase = rng.uniform(0.0, 2 * np.pi, size=amp.shape)
    z = np.fft.irfft2(amp * np.exp(1j * phase), s=(ny, nx))
    z = z / np.sqrt(np.mean(z * z))
    return z.reshape(-1)


def draws(cfg, seed=0):
    """Raw draws for one problem: x_true, xi (n), eta (n_t, n_obs).  BVE draws the
    truth's phases first."""
    rng = np.random.default_rng(seed)
    x_true = bve_truth(cfg, rng) if cfg.get('model') == 'bve' else truth(cfg)
    xi = rng.standard_normal(cfg['n'])
    eta = rng.standard_normal((n_t(cfg), n_obs(cfg)))
    return dict(x_true=x_true, xi=xi, eta=eta)


def omega(n, ell, seed=1000):
    """Gaussian test matrix Omega (n x ell), row-major (grid point major)."""
    return np.random.default_rng(seed).standard_normal((n, ell))


def unit_vector(n, seed=2000):
    w = np.random.default_rng(seed).standard_normal(n)
    return w / np.linalg.norm(w)


def batch_configs(nprob=64, seed=0, n_lo=256, n_hi=4096, N_lo=50, N_hi=500, ell=32):
    """Uneven batch: n = round(exp(U[ln n_lo, ln n_hi])), N ~ U{N_lo..N_hi};
    observation layout and prior as in the 128-point workload, dt reduced where
    the configured 1e-3 is outside RK4's stability interval."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss)
    out = []
    for p, child in enumerate(ss.spawn(nprob)):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        N = int(rng.integers(N_lo, N_hi + 1))
        cfg = burgers_config(n, N, 4, 10, dt_cfg=1e-3, ell=ell, name=f'batch-{p}')
        cfg['seed'] = int(child.generate_state(1)[0])
        out.append(cfg)
    return out
