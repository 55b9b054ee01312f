"""Oracle: periodic viscous Burgers model, RK4, and its discrete RK TLM / ADJ.

Test infrastructure only (see ``oracle/__init__``).

The model is u_t + u u_x = nu u_xx (Sec. 5.1, eq. (1dburgers)) discretised with
second-order central differences on the periodic grid x_j = j/n, j = 0..n-1
(advective form, nodes at j/n), and advanced with the classical four-stage
Runge-Kutta method.  The paper uses Dirichlet walls and a third-order TVD RK
scheme; the periodic RK4 variant is the measured workload and is recorded as a
reading in the design notes.

The tangent-linear and adjoint are the *discrete* Runge-Kutta TLM and adjoint
(Sec. 2.1, last paragraph; Sec. 5.1 names the discrete Runge-Kutta versions),
i.e. the exact linearisation of the stage recurrences and its exact transpose,
not a discretisation of the continuous adjoint PDE.

Arrays: a state is shape (n,); a block of k perturbations is shape (n, k)
(grid point major, vector minor).  All float64.
"""
import numpy as np

# classical RK4 tableau: stage offsets and weights
RK4_C = (0.0, 0.5, 0.5, 1.0)
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)


def _shift(a, s):
    """a[(j + s) mod n] along axis 0."""
    return np.roll(a, -s, axis=0)


def rhs(u, nu, dx):
    """Semi-discrete right-hand side f(u)_j = -u_j (u_{j+1}-u_{j-1})/(2dx)
    + nu (u_{j+1} - 2u_j + u_{j-1})/dx^2 (eq. (1dburgers), central FD)."""
    up, um = _shift(u, 1), _shift(u, -1)
    return -u * (up - um) / (2.0 * dx) + nu * (up - 2.0 * u + um) / (dx * dx)


def jac(Y, d, nu, dx):
    """J(Y) d: derivative of rhs at Y applied to d (d is (n,) or (n,k))."""
    Yc = Y if d.ndim == 1 else Y[:, None]
    Yp, Ym = _shift(Y, 1), _shift(Y, -1)
    DY = (Yp - Ym) / (2.0 * dx)
    DYc = DY if d.ndim == 1 else DY[:, None]
    dp, dm = _shift(d, 1), _shift(d, -1)
    return -d * DYc - Yc * (dp - dm) / (2.0 * dx) + nu * (dp - 2.0 * d + dm) / (dx * dx)


def jac_t(Y, l, nu, dx):
    """J(Y)^T l: the exact transpose of ``jac`` (row j of J(Y) has entries
    -DY_j - 2nu/dx^2 on the diagonal, -Y_j/(2dx) + nu/dx^2 at j+1 and
    +Y_j/(2dx) + nu/dx^2 at j-1)."""
    Yp, Ym = _shift(Y, 1), _shift(Y, -1)
    DY = (Yp - Ym) / (2.0 * dx)
    if l.ndim == 2:
        DY = DY[:, None]
        Y = Y[:, None]
    Yl = Y * l
    lp, lm = _shift(l, 1), _shift(l, -1)
    return -DY * l + (_shift(Yl, 1) - _shift(Yl, -1)) / (2.0 * dx) + nu * (lp - 2.0 * l + lm) / (dx * dx)


def rk4_stages(u, h, nu, dx):
    """Nonlinear RK4 stage states Y1..Y4 of the step starting at u."""
    Y1 = u
    K1 = rhs(Y1, nu, dx)
    Y2 = u + 0.5 * h * K1
    K2 = rhs(Y2, nu, dx)
    Y3 = u + 0.5 * h * K2
    K3 = rhs(Y3, nu, dx)
    Y4 = u + h * K3
    return Y1, Y2, Y3, Y4


def rk4_step(u, h, nu, dx):
    """One classical RK4 step of the semi-discrete model (eq. (model))."""
    K1 = rhs(u, nu, dx)
    K2 = rhs(u + 0.5 * h * K1, nu, dx)
    K3 = rhs(u + 0.5 * h * K2, nu, dx)
    K4 = rhs(u + h * K3, nu, dx)
    return u + h * (K1 / 6.0 + K2 / 3.0 + K3 / 3.0 + K4 / 6.0)


def fwd(u0, h, nsteps, nu, dx):
    """Nonlinear trajectory u_0..u_N (eq. (model)); returns array (N+1, n)."""
    traj = np.empty((nsteps + 1,) + np.shape(u0), dtype=np.result_type(u0, np.float64))
    traj[0] = u0
    for s in range(nsteps):
        traj[s + 1] = rk4_step(traj[s], h, nu, dx)
    return traj


def tlm_step(u, d, h, nu, dx):
    """Discrete RK4 tangent-linear step around base state u: the exact
    linearisation of the four stage recurrences (Sec. 2.1, discrete RK TLM)."""
    Y1, Y2, Y3, Y4 = rk4_stages(u, h, nu, dx)
    dK1 = jac(Y1, d, nu, dx)
    dK2 = jac(Y2, d + 0.5 * h * dK1, nu, dx)
    dK3 = jac(Y3, d + 0.5 * h * dK2, nu, dx)
    dK4 = jac(Y4, d + h * dK3, nu, dx)
    return d + h * (dK1 / 6.0 + dK2 / 3.0 + dK3 / 3.0 + dK4 / 6.0)


def adj_step(u, lam, h, nu, dx):
    """Discrete RK4 adjoint step: the exact transpose of ``tlm_step`` taken in
    reverse stage order (Sandu's discrete Runge-Kutta adjoint, Sec. 2.1)."""
    Y1, Y2, Y3, Y4 = rk4_stages(u, h, nu, dx)
    out = lam.copy()
    mu4 = h / 6.0 * lam
    th4 = jac_t(Y4, mu4, nu, dx)
    out += th4
    mu3 = h / 3.0 * lam + h * th4
    th3 = jac_t(Y3, mu3, nu, dx)
    out += th3
    mu2 = h / 3.0 * lam + 0.5 * h * th3
    th2 = jac_t(Y2, mu2, nu, dx)
    out += th2
    mu1 = h / 6.0 * lam + 0.5 * h * th2
    th1 = jac_t(Y1, mu1, nu, dx)
    out += th1
    return out


def tlm(traj, d0, h, nu, dx, obs_steps):
    """Propagate perturbation(s) d0 along the trajectory; return the list of
    states delta u_{s_i} at the observation steps (increasing order)."""
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
    """Adjoint sweep: lambda = 0 at the end of the window; at each observation
    step s_i the forcing for that step is added before the step s_i-1 -> s_i is
    transposed; returns lambda_0.  ``forcings[i]`` is a full state-space array
    (already mapped through O^T) for step obs_steps[i]."""
    steps = [int(s) for s in obs_steps]
    last = max(steps) if steps else 0
    shape = np.shape(forcings[0])
    lam = np.zeros(shape, dtype=np.float64)
    f_at = {s: forcings[i] for i, s in enumerate(steps)}
    for s in range(last, 0, -1):
        if s in f_at:
            lam = lam + f_at[s]
        lam = adj_step(traj[s - 1], lam, h, nu, dx)
    return lam


# ---------------------------------------------------------------------------
# Scalar-loop variant (small n only) used to cross-check the vectorised code.
# ---------------------------------------------------------------------------

def rhs_loop(u, nu, dx):
    n = len(u)
    f = [0.0] * n
    for j in range(n):
        up, um = u[(j + 1) % n], u[(j - 1) % n]
        f[j] = -u[j] * (up - um) / (2.0 * dx) + nu * (up - 2.0 * u[j] + um) / (dx * dx)
    return np.array(f)


def jac_loop(Y, d, nu, dx):
    n = len(Y)
    out = [0.0] * n
    for j in range(n):
        Yp, Ym = Y[(j + 1) % n], Y[(j - 1) % n]
        dp, dm = d[(j + 1) % n], d[(j - 1) % n]
        out[j] = (-d[j] * (Yp - Ym) / (2.0 * dx) - Y[j] * (dp - dm) / (2.0 * dx)
                  + nu * (dp - 2.0 * d[j] + dm) / (dx * dx))
    return np.array(out)


def jac_matrix_loop(Y, nu, dx):
    """Dense J(Y) assembled entry by entry (row j, columns j-1, j, j+1)."""
    n = len(Y)
    J = np.zeros((n, n))
    for j in range(n):
        Yp, Ym = Y[(j + 1) % n], Y[(j - 1) % n]
        J[j, j] += -(Yp - Ym) / (2.0 * dx) - 2.0 * nu / (dx * dx)
        J[j, (j + 1) % n] += -Y[j] / (2.0 * dx) + nu / (dx * dx)
        J[j, (j - 1) % n] += Y[j] / (2.0 * dx) + nu / (dx * dx)
    return J
