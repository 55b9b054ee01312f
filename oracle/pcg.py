"""Oracle: preconditioned conjugate gradients on (I + H) dx = b.

Test infrastructure only (see ``oracle/__init__``).

Follows Sec. 2.2.2 (SketchPrec, eq. (pcgsystem)): CG on the first-level
preconditioned GN system, preconditioned by the limited-memory preconditioner of
eq. (woodbury) (or by the identity: the paper's Prec_Gamma).  Readings: x_0 = 0;
the loop stops when the recurrence residual satisfies ||r_k||_2 <= rtol ||b||_2
(Sec. 5 stops PCG on a prescribed relative residual); every iteration costs exactly one (I + H) product
(online TLM = number of PCG iterations, Tables 2 and 4).
"""
import numpy as np


def pcg(op, b, prec=None, rtol=1e-6, maxit=None):
    """Returns (x, info) with info = dict(iters, relres, converged, history)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    if maxit is None:
        maxit = n
    x = np.zeros_like(b)
    r = b.copy()
    z = prec(r) if prec is not None else r.copy()
    p = z.copy()
    rz = float(r @ z)
    bnorm = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r))]
    it = 0
    converged = bnorm == 0.0 or hist[-1] <= rtol * bnorm
    while not converged and it < maxit:
        q = op(p)
        alpha = rz / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(float(np.linalg.norm(r)))
        if hist[-1] <= rtol * bnorm:
            converged = True
            break
        z = prec(r) if prec is not None else r.copy()
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    relres = hist[-1] / bnorm if bnorm > 0 else 0.0
    return x, dict(iters=it, relres=relres, converged=converged, history=hist)
