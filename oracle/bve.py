"""Oracle: periodic barotropic vorticity model, RK4, and its discrete RK TLM / ADJ.

Test infrastructure only (see ``oracle/__init__``).

Model (the measured workload; the paper's gyre configuration with Dirichlet walls,
forcing and Rossby term is not reproduced -- Sec. 5.2 describes it):
    zeta_t + J(psi, zeta) = nu lap(zeta),   lap(psi) = zeta
on the periodic unit square with an nx x ny grid, spacing d = 1/nx = 1/ny.
J(a, b) = a_x b_y - a_y b_x is discretised with Arakawa's energy- and
enstrophy-conserving Jacobian J_A = (J++ + J+x + Jx+)/3; lap(zeta) with the
5-point stencil; psi = L zeta with the spectral inverse Laplacian
(psi_hat = -zeta_hat / |k|^2, |k|^2 = (2 pi)^2 (kx^2 + ky^2), zero mode 0), which
is a library FFT step here.  Fields are arrays (ny, nx) (row j = y index); the
flattened state is j*nx + i.

The TLM of the RHS f(zeta) = -J_A(L zeta, zeta) + nu lap(zeta) is
    df = -J_A(L dz, zeta) - J_A(L zeta, dz) + nu lap(dz)
and its adjoint, using the total antisymmetry of Arakawa's trilinear form
sum c J_A(a, b) (pinned by the tests against an explicitly transposed matrix):
    df^T lam = -L J_A(zeta, lam) + J_A(L zeta, lam) + nu lap(lam).
RK4 TLM/ADJ wrap these stage Jacobians exactly as for Burgers (discrete RK adjoint).
"""
import numpy as np


def _sh(a, di, dj):
    """a[j + dj, i + di] (periodic) for arrays (..., ny, nx) or (ny, nx, k)."""
    return np.roll(np.roll(a, -dj, axis=0), -di, axis=1)


def arakawa(a, b, d):
    """Arakawa Jacobian J_A(a, b) for fields (ny, nx[, k]) on spacing d."""
    ap, am = _sh(a, 1, 0), _sh(a, -1, 0)       # a_{i+1,j}, a_{i-1,j}
    aN, aS = _sh(a, 0, 1), _sh(a, 0, -1)       # a_{i,j+1}, a_{i,j-1}
    bp, bm = _sh(b, 1, 0), _sh(b, -1, 0)
    bN, bS = _sh(b, 0, 1), _sh(b, 0, -1)
    bpN, bpS = _sh(b, 1, 1), _sh(b, 1, -1)
    bmN, bmS = _sh(b, -1, 1), _sh(b, -1, -1)
    apN, apS = _sh(a, 1, 1), _sh(a, 1, -1)
    amN, amS = _sh(a, -1, 1), _sh(a, -1, -1)
    jpp = (ap - am) * (bN - bS) - (aN - aS) * (bp - bm)
    jpx = ap * (bpN - bpS) - am * (bmN - bmS) - aN * (bpN - bmN) + aS * (bpS - bmS)
    jxp = bN * (apN - amN) - bS * (apS - amS) - bp * (apN - apS) + bm * (amN - amS)
    return (jpp + jpx + jxp) / (12.0 * d * d)


def lap5(a, d):
    return (_sh(a, 1, 0) + _sh(a, -1, 0) + _sh(a, 0, 1) + _sh(a, 0, -1) - 4.0 * a) / (d * d)


def kk2(ny, nx):
    ky = np.fft.fftfreq(ny, d=1.0 / ny)
    kx = np.fft.fftfreq(nx, d=1.0 / nx)
    return (2 * np.pi) ** 2 * (ky[:, None] ** 2 + kx[None, :] ** 2)


def inv_lap(z):
    """Spectral inverse Laplacian (zero mean): psi with lap(psi) = z - mean(z)."""
    ny, nx = z.shape[:2]
    k2 = kk2(ny, nx)
    with np.errstate(divide='ignore'):
        m = np.where(k2 > 0, -1.0 / k2, 0.0)
    if z.ndim == 3:
        m = m[:, :, None]
    if not np.isrealobj(z):
        # L is a real operator: apply it to both parts so that the FFT's roundoff in
        # one part does not leak into the other (keeps complex-step derivatives exact)
        return inv_lap(z.real) + 1j * inv_lap(z.imag)
    return np.fft.ifft2(np.fft.fft2(z, axes=(0, 1)) * m, axes=(0, 1)).real


def rhs(z, nu, d):
    return -arakawa(inv_lap(z), z, d) + nu * lap5(z, d)


def jac(Y, dz, nu, d):
    """Derivative of rhs at Y applied to dz (fields (ny, nx[, k]))."""
    Yb = Y if dz.ndim == 2 else Y[:, :, None]
    psi = inv_lap(Y)
    psib = psi if dz.ndim == 2 else psi[:, :, None]
    return -arakawa(inv_lap(dz), Yb, d) - arakawa(psib, dz, d) + nu * lap5(dz, d)


def jac_t(Y, lam, nu, d):
    """Transpose of ``jac`` at Y (identity-based form, see module docstring)."""
    Yb = Y if lam.ndim == 2 else Y[:, :, None]
    psi = inv_lap(Y)
    psib = psi if lam.ndim == 2 else psi[:, :, None]
    return -inv_lap(arakawa(Yb, lam, d)) + arakawa(psib, lam, d) + nu * lap5(lam, d)


class BVEModel:
    """Periodic BVE on an nx x ny grid, RK4 with step dt; states flattened j*nx+i."""

    def __init__(self, nx, ny, nu, dt):
        self.nx, self.ny, self.nu, self.dt = int(nx), int(ny), float(nu), float(dt)
        self.d = 1.0 / self.nx

    @property
    def n(self):
        return self.nx * self.ny

    def _f(self, v):
        return v.reshape((self.ny, self.nx) + v.shape[1:])

    def _u(self, a):
        return a.reshape((self.n,) + a.shape[2:])

    def stages(self, z):
        h, nu, d = self.dt, self.nu, self.d
        Y1 = z
        K1 = rhs(Y1, nu, d)
        Y2 = z + 0.5 * h * K1
        K2 = rhs(Y2, nu, d)
        Y3 = z + 0.5 * h * K2
        K3 = rhs(Y3, nu, d)
        Y4 = z + h * K3
        return Y1, Y2, Y3, Y4

    def step(self, z):
        h, nu, d = self.dt, self.nu, self.d
        K1 = rhs(z, nu, d)
        K2 = rhs(z + 0.5 * h * K1, nu, d)
        K3 = rhs(z + 0.5 * h * K2, nu, d)
        K4 = rhs(z + h * K3, nu, d)
        return z + h * (K1 / 6.0 + K2 / 3.0 + K3 / 3.0 + K4 / 6.0)

    def fwd(self, x0, nsteps):
        z = self._f(np.asarray(x0, dtype=np.result_type(x0, np.float64)))
        out = np.empty((nsteps + 1, self.n), dtype=z.dtype)
        out[0] = self._u(z)
        for s in range(nsteps):
            z = self.step(z)
            out[s + 1] = self._u(z)
        return out

    def tlm_step(self, z, dz):
        h, nu, d = self.dt, self.nu, self.d
        Y1, Y2, Y3, Y4 = self.stages(z)
        k1 = jac(Y1, dz, nu, d)
        k2 = jac(Y2, dz + 0.5 * h * k1, nu, d)
        k3 = jac(Y3, dz + 0.5 * h * k2, nu, d)
        k4 = jac(Y4, dz + h * k3, nu, d)
        return dz + h * (k1 / 6.0 + k2 / 3.0 + k3 / 3.0 + k4 / 6.0)

    def adj_step(self, z, lam):
        h, nu, d = self.dt, self.nu, self.d
        Y1, Y2, Y3, Y4 = self.stages(z)
        out = lam.copy()
        mu4 = h / 6.0 * lam
        th4 = jac_t(Y4, mu4, nu, d)
        out += th4
        mu3 = h / 3.0 * lam + h * th4
        th3 = jac_t(Y3, mu3, nu, d)
        out += th3
        mu2 = h / 3.0 * lam + 0.5 * h * th3
        th2 = jac_t(Y2, mu2, nu, d)
        out += th2
        mu1 = h / 6.0 * lam + 0.5 * h * th2
        th1 = jac_t(Y1, mu1, nu, d)
        out += th1
        return out

    def tlm(self, traj, d0, obs_steps):
        want = set(int(s) for s in obs_steps)
        last = max(want) if want else 0
        dz = self._f(np.array(d0, dtype=np.float64, copy=True))
        res = {}
        for s in range(last):
            dz = self.tlm_step(self._f(traj[s]), dz)
            if s + 1 in want:
                res[s + 1] = self._u(dz).copy()
        return [res[int(s)] for s in obs_steps]

    def adj(self, traj, forcings, obs_steps):
        steps = [int(s) for s in obs_steps]
        last = max(steps) if steps else 0
        lam = np.zeros((self.ny, self.nx) + np.shape(forcings[0])[1:])
        f_at = {s: self._f(forcings[i]) for i, s in enumerate(steps)}
        for s in range(last, 0, -1):
            if s in f_at:
                lam = lam + f_at[s]
            lam = self.adj_step(self._f(traj[s - 1]), lam)
        return self._u(lam)

    def obs_index(self, stride):
        j = np.arange(0, self.ny, stride)
        i = np.arange(0, self.nx, stride)
        return (j[:, None] * self.nx + i[None, :]).reshape(-1)

    def bhalf(self, V, sigma_b, L):
        from .prior import bhalf_2d
        return bhalf_2d(V, self.nx, self.ny, sigma_b, L)
