"""Oracle: randomized low-rank approximations of the data-misfit Hessian and the
limited-memory preconditioner they define.

Test infrastructure only (see ``oracle/__init__``).

  * RandSVD      Sec. 3.1.1, Alg. 1 (randsvd): H = A^T A approximated by the
                 projection A^T Q Q^T A onto the range of A Omega
  * Nystrom      Sec. 3.1.1, Alg. 2 (nystrom): the shifted Nystrom approximant
                 (H Omega)(Omega^T H Omega)^{-1}(H Omega)^T (Tropp et al.)
  * LMP          eq. (woodbury): (I + V L V^T)^{-1} = I - V (L^{-1} + I)^{-1} V^T
  * W-form       Remark 1, eq. (randsvdsv): (I + W^T W)^{-1} = I - W^T (I + W W^T)^{-1} W
  * adaptive     Sec. 3.1.2, Alg. 4 (randsvd_adaptive) with the test kappa_sk of
                 eq. (condtext); the Nystrom form (nystrom_adaptive)
  * SingleView   Sec. 3.1.1, Alg. 3 (singleview), the oblique-projector
                 approximation of eq. (singleviewlr); adaptive form Alg. 5
                 (singleview_adaptive) with the QR update of Alg. 6 (qr_update)

Readings: no truncation (target rank r = l); machine epsilon of Nystrom's shift
is that of the precision Y was computed in (2^-52 for float64, 2^-23 for
float32); ||Y||_2 is the exact spectral norm; if the Cholesky factorisation of
the shifted core matrix fails the shift is multiplied by 10 (at most 3 times);
D = lambda / (1 + lambda) is the diagonal (Lambda^{-1} + I)^{-1} written so that
lambda = 0 is allowed.
"""
import numpy as np
from scipy.linalg import solve_triangular

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -23


class NotSPDError(RuntimeError):
    pass


def nystrom(H_apply, Omega, eps=EPS64, max_retries=3):
    """Nystrom approximation of H from the sketch H Omega (Sec. 3.1.1, Alg. 2):
    returns (V_hat (n x l), lambda_hat (l,), nu)."""
    Omega = np.asarray(Omega, dtype=np.float64)
    return nystrom_from_sketch(Omega, H_apply(Omega), eps, max_retries)


def nystrom_from_sketch(Omega, Y0, eps=EPS64, max_retries=3):
    """Nystrom approximation given the sketch Y0 = H Omega.

    The approximant is built for the shifted operator H + nu I, whose sketch is
    Y0 + nu Omega, and the shift is removed from its eigenvalues afterwards:

        H_nu_hat = Y_nu (Omega^T Y_nu)^{-1} Y_nu^T,   Y_nu = Y0 + nu Omega,
        nu = sqrt(n) eps ||Y0||_2.

    With the Cholesky factor C_nu = L L^T of the (symmetrised) core
    C_nu = Omega^T Y_nu, H_nu_hat = B B^T for B = Y_nu L^{-T}; the thin SVD
    B = V Sigma U^T gives the eigenpairs (V, Sigma^2) of H_nu_hat, and the
    approximation of H keeps V with lambda = max(0, Sigma^2 - nu).  A core that
    is not numerically positive definite is retried with the shift multiplied
    by 10, at most ``max_retries`` times."""
    Omega = np.asarray(Omega, dtype=np.float64)
    n, ell = Omega.shape
    nu = np.sqrt(n) * eps * np.linalg.norm(Y0, 2)
    for _ in range(max_retries + 1):
        Y = Y0 + nu * Omega
        C = Omega.T @ Y
        try:
            L = np.linalg.cholesky(0.5 * (C + C.T))
        except np.linalg.LinAlgError:
            nu *= 10.0
            continue
        Bt = solve_triangular(L, Y.T, lower=True)         # B^T = L^{-1} Y_nu^T
        _, S, Vt = np.linalg.svd(Bt, full_matrices=False)
        lam = np.maximum(0.0, S * S - nu)
        return Vt.T.copy(), lam, nu
    raise NotSPDError("Nystrom core matrix not positive definite after shift retries")


def randsvd(A_apply, AT_apply, Omega):
    """Randomized SVD of A, hence eigendecomposition of H = A^T A (Sec. 3.1.1,
    Alg. 1): with Q an orthonormal basis of range(A Omega), H is approximated
    by A^T Q Q^T A = W^T W for W = Q^T A, whose thin SVD W = U Sigma V^T gives
    H_hat = V Sigma^2 V^T.  A_apply maps (n, l) -> (m, l); AT_apply maps
    (m, l) -> (n, l).  Returns (V_hat, lambda_hat)."""
    Omega = np.asarray(Omega, dtype=np.float64)
    Q, _ = np.linalg.qr(A_apply(Omega))                   # Householder thin QR
    Wt = AT_apply(Q)                                      # W^T = A^T Q
    _, S, Vt = np.linalg.svd(Wt.T, full_matrices=False)
    return Vt.T.copy(), S * S


def randsvd_W(A_apply, AT_apply, Omega):
    """The factor W = Q^T A (l x n) of the randomized SVD, H_hat = W^T W, without
    its SVD (the form used by Remark 1)."""
    Y = A_apply(np.asarray(Omega, dtype=np.float64))
    Q, _ = np.linalg.qr(Y)
    return AT_apply(Q).T.copy()


def singleview(A_apply, AT_apply, Omega, Psi):
    """SingleView approximation (Sec. 3.1.1, Alg. 3, eq. (singleviewlr)): from
    the independent sketches Y = A Omega (m x l1) and Z = A^T Psi (n x l2),
    A is approximated by Q_Y M^+ Z^T with Q_Y an orthonormal basis of range(Y)
    and M = Psi^T Q_Y = Q_M R_M (thin QR), so M^+ = R_M^{-1} Q_M^T.  Then
    H = A^T A is approximated by W^T W with W = R_M^{-1} (Z Q_M)^T, whose thin
    SVD gives H_hat = V Sigma^2 V^T.  Thin QRs by Householder; M has full
    column rank for Gaussian Psi with l2 >= l1."""
    Omega = np.asarray(Omega, dtype=np.float64)
    Psi = np.asarray(Psi, dtype=np.float64)
    Y = A_apply(Omega)
    Z = AT_apply(Psi)
    Qy, _ = np.linalg.qr(Y)
    Qm, Rm = np.linalg.qr(Psi.T @ Qy)
    W = solve_triangular(Rm, (Z @ Qm).T, lower=False)
    _, S, Vt = np.linalg.svd(W, full_matrices=False)
    return Vt.T.copy(), S * S


def kappa_sk(H_apply, W, v):
    """eq. (condtext): |(I + H)(I + H_hat)^{-1} v|_2 with H_hat = W^T W, the inverse
    by eq. (randsvdsv); v is normalised here (a unit test vector)."""
    v = np.asarray(v, dtype=np.float64)
    v = v / np.linalg.norm(v)
    u = woodbury_W_apply(W, v)
    return float(np.linalg.norm(u + H_apply(u[:, None])[:, 0]))


def randsvd_adaptive(A_apply, AT_apply, H_apply, Omegas, v, eps_sk):
    """Alg. 4 (adaptive RandSVD).  Omegas is the sequence of Gaussian blocks the
    algorithm draws (the first of width l, then blocks of width l_hat); v the
    test vector of kappa_sk (the same at every evaluation).  The loop enlarges
    the sketch while kappa_sk > eps_sk and blocks remain (the caller's cap on
    l).  Returns (V_hat, lambda_hat, kappas) with one kappa_sk per evaluation.
    Readings: the new block is orthogonalised against the accumulated Q twice
    (classical Gram-Schmidt with one re-orthogonalisation: the optional extra
    Gram-Schmidt passes the algorithm allows, always taken); thin QR by
    Householder."""
    Om = np.asarray(Omegas[0], dtype=np.float64)
    Y = A_apply(Om)                                        # forward pass Y = A Omega
    Qh, _ = np.linalg.qr(Y)                                # thin QR
    Wt = AT_apply(Qh)                                      # W^T = A^T Q_hat
    Q = np.zeros((Y.shape[0], 0))
    kappas = [kappa_sk(H_apply, Wt.T, v)]
    for blk in Omegas[1:]:
        if kappas[-1] <= eps_sk:
            break
        Q = np.hstack([Q, Qh])                             # append Q_hat
        Y = A_apply(np.asarray(blk, dtype=np.float64))     # forward pass on the new block
        for _ in range(2):
            Y = Y - Q @ (Q.T @ Y)                          # orthogonalise against Q
        Qh, _ = np.linalg.qr(Y)
        Wt = np.hstack([Wt, AT_apply(Qh)])                 # W <- [W; W_hat]
        kappas.append(kappa_sk(H_apply, Wt.T, v))
    _, S, Vt = np.linalg.svd(Wt.T, full_matrices=False)    # thin SVD of W
    return Vt.T.copy(), S * S, kappas


def qr_update(A1, A2, B1, B2, Q1, R1):
    """Thin QR of the stacked product [A1; A2] [B1 B2] given the thin QR
    Q1 R1 = A1 B1 (Sec. 3.1.2, Alg. 6; B1, B2 with orthonormal columns).

    The first block column [A1 B1; A2 B1] = diag(Q1, Q2) [R1; R2] once
    A2 B1 = Q2 R2 is factored, and one more QR [R1; R2] = Q3' R3 gives its thin
    QR Q3 R3 with Q3 = diag(Q1, Q2) Q3'.  The second block column P1 = [A1; A2] B2
    is split into its component T = Q3^T P1 in range(Q3) and the remainder
    P2 = P1 - Q3 T = Q4 R4, so [Q3 Q4] [[R3, T], [0, R4]] is the thin QR of the
    whole.  Thin QRs by Householder; A2 B1 may be wider than tall, whose reduced
    QR has a trapezoidal R.  Returns (Q5, R5)."""
    Q2, R2 = np.linalg.qr(A2 @ B1)
    Q3s, R3 = np.linalg.qr(np.vstack([R1, R2]))
    k1 = R1.shape[0]
    Q3 = np.vstack([Q1 @ Q3s[:k1], Q2 @ Q3s[k1:]])
    P1 = np.vstack([A1, A2]) @ B2
    T = Q3.T @ P1
    Q4, R4 = np.linalg.qr(P1 - Q3 @ T)
    Q5 = np.hstack([Q3, Q4])
    R5 = np.block([[R3, T], [np.zeros((R4.shape[0], R3.shape[1])), R4]])
    return Q5, R5


def singleview_adaptive(A_apply, AT_apply, H_apply, Omegas, Psis, v, eps_sk, qr='direct'):
    """Alg. 5 (adaptive SingleView).  Omegas / Psis are the Gaussian blocks the
    algorithm draws, pairwise (first (l1, l2), then (l1_hat, l2_hat) per
    extension); v the test vector of kappa_sk.  While kappa_sk > eps_sk and
    blocks remain: Y_hat = A Omega_hat and Z_hat = A^T Psi_hat, Y_hat is
    orthogonalised twice against Q_Y and factored, Q_Y, Psi and Z grow by the
    new blocks, M = Psi^T Q_Y = Q_M R_M is refactored (qr='direct') or updated
    by Alg. 6 (qr='update'), and W = R_M^{-1} (Z Q_M)^T is formed anew.
    Readings: the algorithm's lines that form A^T Q_hat and stack it onto W are
    RandSVD steps that do not fit the SingleView construction (whose W comes
    from Z and the factors of M, and which draws Psi_hat without sweeping it);
    they are read as the co-range sketch Z_hat = A^T Psi_hat followed by the
    SingleView W.  kappa_sk by eq. (condtext) with H_hat = W^T W and eq.
    (randsvdsv).  Returns (V_hat, lambda_hat, kappas)."""
    Psi = np.asarray(Psis[0], dtype=np.float64)
    Y = A_apply(np.asarray(Omegas[0], dtype=np.float64))  # both sketches
    Z = AT_apply(Psi)
    Qy, _ = np.linalg.qr(Y)
    Qm, Rm = np.linalg.qr(Psi.T @ Qy)
    W = solve_triangular(Rm, (Z @ Qm).T, lower=False)
    kappas = [kappa_sk(H_apply, W, v)]
    for Om_h, Psi_h in zip(Omegas[1:], Psis[1:]):
        if kappas[-1] <= eps_sk:
            break
        Psi_h = np.asarray(Psi_h, dtype=np.float64)
        Y = A_apply(np.asarray(Om_h, dtype=np.float64))   # new range and co-range blocks
        Zh = AT_apply(Psi_h)
        for _ in range(2):
            Y = Y - Qy @ (Qy.T @ Y)                        # orthogonalise against Q_Y
        Qh, _ = np.linalg.qr(Y)
        if qr == 'update':
            Qm, Rm = qr_update(Psi.T, Psi_h.T, Qy, Qh, Qm, Rm)
        Qy = np.hstack([Qy, Qh])
        Psi = np.hstack([Psi, Psi_h])
        Z = np.hstack([Z, Zh])
        if qr == 'direct':
            Qm, Rm = np.linalg.qr(Psi.T @ Qy)
        W = solve_triangular(Rm, (Z @ Qm).T, lower=False)
        kappas.append(kappa_sk(H_apply, W, v))
    _, S, Vt = np.linalg.svd(W, full_matrices=False)
    return Vt.T.copy(), S * S, kappas


def nystrom_adaptive(H_apply, Omegas, v, eps_sk, eps=EPS64):
    """Adaptive Nystrom (Sec. 3.1.2).  The paper gives the loop for RandSVD
    (Alg. 4) and calls the Nystrom form similar; read as: each round appends the
    next Gaussian block of ``Omegas`` to Omega, sweeps only that block
    (H Omega is formed column by column) and forms Alg. 2 on every column so
    far; kappa_sk of eq. (condtext) uses (I + H_hat)^{-1} by eq. (woodbury);
    the loop stops once kappa_sk <= eps_sk or no block remains.
    Returns (V_hat, lambda_hat, nu, kappas)."""
    vu = np.asarray(v, dtype=np.float64)
    vu = vu / np.linalg.norm(vu)
    cols, Ys, kappas = [], [], []
    for blk in Omegas:
        if kappas and kappas[-1] <= eps_sk:
            break
        blk = np.asarray(blk, dtype=np.float64)
        cols.append(blk)
        Ys.append(H_apply(blk))                            # sweep of the new block only
        V, lam, nu = nystrom_from_sketch(np.hstack(cols), np.hstack(Ys), eps)
        u = lmp_apply(V, lam, vu)
        kappas.append(float(np.linalg.norm(u + H_apply(u[:, None])[:, 0])))
    return V, lam, nu, kappas


def lmp_diag(lam):
    """(Lambda^{-1} + I)^{-1} = lambda / (1 + lambda)."""
    lam = np.asarray(lam, dtype=np.float64)
    return lam / (1.0 + lam)


def lmp_apply(V, lam, r):
    """(I + V diag(lam) V^T)^{-1} r via eq. (woodbury); r is (n,) or (n, k)."""
    D = lmp_diag(lam)
    t = V.T @ r
    t = D * t if t.ndim == 1 else D[:, None] * t
    return r - V @ t


def woodbury_W_apply(W, r):
    """(I + W^T W)^{-1} r via eq. (randsvdsv), using an l x l Cholesky."""
    ell = W.shape[0]
    Lc = np.linalg.cholesky(np.eye(ell) + W @ W.T)
    t = W @ r
    t = solve_triangular(Lc, t, lower=True)
    t = solve_triangular(Lc.T, t, lower=False)
    return r - W.T @ t


def hhat_apply(V, lam, X):
    """H_hat X = V diag(lam) V^T X."""
    t = V.T @ X
    t = lam * t if t.ndim == 1 else lam[:, None] * t
    return V @ t
