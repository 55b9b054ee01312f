"""Oracle: the paper's Burgers setup -- homogeneous Dirichlet walls, second-order
central differences, the three-stage TVD Runge-Kutta method -- with its discrete
RK TLM and ADJ.

Test infrastructure only (see ``oracle/__init__``).

Sec. 5.1: u_t + u u_x = nu u_xx on (0, 1), u(t, 0) = u(t, 1) = 0, central
second-order differences on a uniform mesh, time stepping by the third-order
TVD Runge-Kutta scheme of Gottlieb and Shu (1998), whose Shu-Osher form is

    w1 = u + h f(u)
    w2 = 3/4 u + 1/4 (w1 + h f(w1))
    u+ = 1/3 u + 2/3 (w2 + h f(w2)).

Grid: the n interior nodes x_j = (j + 1) dx, dx = 1/(n + 1), j = 0..n-1 (the
paper's n = 399 gives dx = 0.0025); the wall values enter the stencils as zeros.

The tangent-linear and adjoint are the discrete ones: the exact linearisation
of the three stage recurrences and its exact transpose in reverse stage order.
Arrays: a state is (n,); a block of k perturbations is (n, k).  Float64.
"""
import numpy as np


def _up(a):
    """a[j + 1] with the wall value 0 past the last node (axis 0)."""
    out = np.zeros_like(a)
    out[:-1] = a[1:]
    return out


def _dn(a):
    """a[j - 1] with the wall value 0 before the first node (axis 0)."""
    out = np.zeros_like(a)
    out[1:] = a[:-1]
    return out


def rhs(u, nu, dx):
    """f(u)_j = -u_j (u_{j+1} - u_{j-1})/(2dx) + nu (u_{j+1} - 2u_j + u_{j-1})/dx^2,
    u_{-1} = u_n = 0 (eq. (1dburgers) with the walls)."""
    up, um = _up(u), _dn(u)
    return -u * (up - um) / (2.0 * dx) + nu * (up - 2.0 * u + um) / (dx * dx)


def jac(Y, d, nu, dx):
    """J(Y) d, the derivative of ``rhs`` at Y applied to d ((n,) or (n, k))."""
    Yc = Y if d.ndim == 1 else Y[:, None]
    DY = (_up(Y) - _dn(Y)) / (2.0 * dx)
    DYc = DY if d.ndim == 1 else DY[:, None]
    dp, dm = _up(d), _dn(d)
    return -d * DYc - Yc * (dp - dm) / (2.0 * dx) + nu * (dp - 2.0 * d + dm) / (dx * dx)


def jac_t(Y, l, nu, dx):
    """J(Y)^T l: row j of J(Y) holds -DY_j - 2nu/dx^2 on the diagonal,
    -Y_j/(2dx) + nu/dx^2 at column j+1 and Y_j/(2dx) + nu/dx^2 at column j-1
    (columns outside 0..n-1 do not exist)."""
    DY = (_up(Y) - _dn(Y)) / (2.0 * dx)
    Yc = Y
    if l.ndim == 2:
        DY = DY[:, None]
        Yc = Y[:, None]
    Yl = Yc * l
    return -DY * l + (_up(Yl) - _dn(Yl)) / (2.0 * dx) + nu * (_up(l) - 2.0 * l + _dn(l)) / (dx * dx)


def rk3_stages(u, h, nu, dx):
    """Stage inputs (u, w1, w2) of one RK3-TVD step."""
    w1 = u + h * rhs(u, nu, dx)
    w2 = 0.75 * u + 0.25 * (w1 + h * rhs(w1, nu, dx))
    return u, w1, w2


def rk3_step(u, h, nu, dx):
    _, w1, w2 = rk3_stages(u, h, nu, dx)
    return u / 3.0 + 2.0 / 3.0 * (w2 + h * rhs(w2, nu, dx))


def fwd(u0, h, nsteps, nu, dx):
    """Trajectory u_0..u_N, shape (N+1, n)."""
    traj = np.empty((nsteps + 1,) + np.shape(u0), dtype=np.float64)
    traj[0] = u0
    for s in range(nsteps):
        traj[s + 1] = rk3_step(traj[s], h, nu, dx)
    return traj


def tlm_step(u, d, h, nu, dx):
    """Linearisation of the three stage recurrences around the base step at u."""
    Y1, Y2, Y3 = rk3_stages(u, h, nu, dx)
    e1 = d + h * jac(Y1, d, nu, dx)
    e2 = 0.75 * d + 0.25 * (e1 + h * jac(Y2, e1, nu, dx))
    return d / 3.0 + 2.0 / 3.0 * (e2 + h * jac(Y3, e2, nu, dx))


def adj_step(u, lam, h, nu, dx):
    """Exact transpose of ``tlm_step``, stages in reverse order."""
    Y1, Y2, Y3 = rk3_stages(u, h, nu, dx)
    mu2 = 2.0 / 3.0 * (lam + h * jac_t(Y3, lam, nu, dx))      # adjoint of e2
    mu1 = 0.25 * (mu2 + h * jac_t(Y2, mu2, nu, dx))           # adjoint of e1
    return lam / 3.0 + 0.75 * mu2 + mu1 + h * jac_t(Y1, mu1, nu, dx)


def tlm(traj, d0, h, nu, dx, obs_steps):
    """Perturbation(s) at the observation steps (increasing order)."""
    want = set(int(s) for s in obs_steps)
    last = max(want) if want else 0
    out = {}
    d = np.array(d0, dtype=np.float64, copy=True)
    for s in range(last):
        d = tlm_step(traj[s], d, h, nu, dx)
        if s + 1 in want:
            out[s + 1] = d.copy()
    return [out[int(s)] for s in obs_steps]


def adj(traj, forcings, h, nu, dx, obs_steps):
    """lambda_0 of the adjoint sweep; forcing i is added at step obs_steps[i]
    before the step into it is transposed (as in the periodic model)."""
    steps = [int(s) for s in obs_steps]
    last = max(steps) if steps else 0
    lam = np.zeros(np.shape(forcings[0]), dtype=np.float64)
    f_at = {s: forcings[i] for i, s in enumerate(steps)}
    for s in range(last, 0, -1):
        if s in f_at:
            lam = lam + f_at[s]
        lam = adj_step(traj[s - 1], lam, h, nu, dx)
    return lam


def jac_matrix_loop(Y, nu, dx):
    """Dense J(Y) assembled entry by entry (small n), walls dropped."""
    n = len(Y)
    J = np.zeros((n, n))
    for j in range(n):
        Yp = Y[j + 1] if j + 1 < n else 0.0
        Ym = Y[j - 1] if j > 0 else 0.0
        J[j, j] = -(Yp - Ym) / (2.0 * dx) - 2.0 * nu / (dx * dx)
        if j + 1 < n:
            J[j, j + 1] = -Y[j] / (2.0 * dx) + nu / (dx * dx)
        if j > 0:
            J[j, j - 1] = Y[j] / (2.0 * dx) + nu / (dx * dx)
    return J
