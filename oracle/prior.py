"""Oracle: Gaussian-kernel background covariance and its symmetric square root.

Test infrastructure only (see ``oracle/__init__``).

The prior covariance of the measured workloads is the periodic Gaussian kernel
B_ij = sigma_b^2 exp(-d_ij^2 / (2 L^2)), d_ij the periodic distance.  The method
needs the symmetric square root Gamma^{1/2} (the factorisation in eq. (Rhalf)
is symmetric: Gamma^{-1/2} (I + A^T A) Gamma^{-1/2}).  B is numerically singular
(its circulant eigenvalues fall below 1e-16 of the largest after a few dozen
Fourier modes), so an eigendecomposition-based square root is ill-conditioned:
sign-flipped roundoff eigenvalues near zero change sqrt(mu) by ~1e-8.

Reading used here: Gamma^{1/2} is the circulant whose kernel is the Gaussian
square-root kernel g(d) = sigma_b a exp(-d^2 / L^2), with a^2 = dx / (L sqrt(pi/2)).
The continuous convolution of g with itself is exactly sigma_b^2 exp(-d^2/(2L^2));
on the grid the aliasing and periodisation errors are exp(-pi^2 L^2/(2 dx^2)) and
exp(-(1/2)^2/L^2), both below double-precision roundoff for every workload here,
so S S = B to roundoff and S is the unique symmetric PSD square root of B up to
roundoff (pinned by tests against the dense matrix and an eigh-based sqrtm).
"""
import numpy as np


def periodic_distance(n, dx):
    d = np.arange(n)
    return np.minimum(d, n - d) * dx


def cov_kernel(n, dx, sigma_b, L):
    """First column c_d of the circulant covariance B."""
    r = periodic_distance(n, dx)
    return sigma_b ** 2 * np.exp(-r * r / (2.0 * L * L))


def sqrt_kernel(n, dx, sigma_b, L):
    """First column g_d of the circulant square root S = Gamma^{1/2}."""
    r = periodic_distance(n, dx)
    a = np.sqrt(dx / (L * np.sqrt(np.pi / 2.0)))
    return sigma_b * a * np.exp(-r * r / (L * L))


def circulant(col):
    """Dense circulant matrix C[i, j] = col[(i - j) mod n]."""
    n = len(col)
    idx = (np.arange(n)[:, None] - np.arange(n)[None, :]) % n
    return col[idx]


def cov_matrix_1d(n, dx, sigma_b, L):
    return circulant(cov_kernel(n, dx, sigma_b, L))


def sqrt_matrix_1d(n, dx, sigma_b, L):
    return circulant(sqrt_kernel(n, dx, sigma_b, L))


def bhalf_1d(V, dx, sigma_b, L):
    """Gamma^{1/2} V for the 1-D prior; V is (n,) or (n, k)."""
    S = sqrt_matrix_1d(V.shape[0], dx, sigma_b, L)
    return S @ V


def bhalf_2d(F, nx, ny, sigma_b, L_cells):
    """Gamma^{1/2} for the separable 2-D prior sigma_b^2 (K_y kron K_x) with K the
    1-D Gaussian kernel in cell units; F is (nx*ny,) or (nx*ny, k) with the grid
    flattened as j*nx + i (x fastest).  Gamma^{1/2} = sigma_b (S_y kron S_x)."""
    Sx = circulant(sqrt_kernel(nx, 1.0, 1.0, L_cells))
    Sy = circulant(sqrt_kernel(ny, 1.0, 1.0, L_cells))
    vec = F.ndim == 1
    G = F.reshape(ny, nx, -1)
    out = np.einsum('ab,bik->aik', Sy, G)
    out = np.einsum('ij,ajk->aik', Sx, out)
    out = sigma_b * out.reshape(nx * ny, -1)
    return out[:, 0] if vec else out


def cov_matrix_2d(nx, ny, sigma_b, L_cells):
    Kx = circulant(cov_kernel(nx, 1.0, 1.0, L_cells))
    Ky = circulant(cov_kernel(ny, 1.0, 1.0, L_cells))
    return sigma_b ** 2 * np.kron(Ky, Kx)


def bhalf_spde_1d(V, alpha, beta):
    """Gamma^{1/2} V for the paper's 1-D prior Gamma = (alpha I - beta Lap*)^{-2}
    (Sec. 5.1, 'Data and Background'; alpha = 0.5, beta = 500 there), i.e. the
    solution X of the tridiagonal system (alpha I - beta Lap*) X = V with Lap*
    the Dirichlet three-point Laplacian tridiag(1, -2, 1) on the interior nodes
    (wall values zero).  Banded solve; V is (n,) or (n, k)."""
    from scipy.linalg import solve_banded
    V = np.asarray(V, dtype=np.float64)
    n = V.shape[0]
    ab = np.zeros((3, n))
    ab[0, 1:] = -beta
    ab[1, :] = alpha + 2.0 * beta
    ab[2, :-1] = -beta
    return solve_banded((1, 1), ab, V)

