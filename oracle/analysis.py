"""Oracle: quantities of the paper's analysis (Sec. 4) used as pins.

Test infrastructure only (see ``oracle/__init__``).

  * intrinsic dimension id_r = sum_{j>r} lambda_j / lambda_{r+1}   Sec. 4.2
  * Psi_H(r, p) = lambda_{r+1} + r/(p-1) sum_{j>r} lambda_j         Thm. (RandSVD)
  * kappa_2 of (I + H_hat)^{-1/2}(I + H)(I + H_hat)^{-1/2}          Thm. (bound_loew)
  * Theta_H(r) = 4 (sum_{j>r} lambda_1 lambda_j)^{1/2} + 4 sum_{j>r} lambda_j
                                                                    Thm. (SingleView)
"""
import numpy as np


def intrinsic_dimension(lam, r):
    lam = np.sort(np.asarray(lam, dtype=np.float64))[::-1]
    return float(np.sum(lam[r:]) / lam[r])


def psi_bound(lam, r, p):
    """Psi_H(r, p) = lambda_{r+1} + r/(p-1) sum_{j>r} lambda_j, the form of the
    definition that stays finite when lambda_{r+1} = 0 (the equal form
    (1 + r/(p-1) id_r) lambda_{r+1} is then 0/0)."""
    lam = np.sort(np.asarray(lam, dtype=np.float64))[::-1]
    return float(lam[r] + r / (p - 1.0) * np.sum(lam[r:]))


def _sym_power(M, power):
    w, U = np.linalg.eigh(0.5 * (M + M.T))
    return (U * w ** power) @ U.T


def precond_kappa(Hd, Hhat):
    """kappa_2((I + Hhat)^{-1/2} (I + Hd) (I + Hhat)^{-1/2}) for dense symmetric
    Hd (the data-misfit Hessian) and Hhat (its approximation)."""
    n = Hd.shape[0]
    Pm = _sym_power(np.eye(n) + Hhat, -0.5)
    K = Pm @ (np.eye(n) + Hd) @ Pm
    w = np.linalg.eigvalsh(0.5 * (K + K.T))
    return float(w[-1] / w[0])


def theta_bound(lam, r):
    """Theta_H(r, p) of the SingleView theorem (l1 = 2r + 1, l2 = 2 l1 + 1)."""
    lam = np.sort(np.asarray(lam, dtype=np.float64))[::-1]
    tail = float(np.sum(lam[r:]))
    return 4.0 * np.sqrt(lam[0] * tail) + 4.0 * tail

