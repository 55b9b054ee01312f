"""Oracle: one Gauss-Newton step of SketchPrec and the sketch-reuse test.

Test infrastructure only (see ``oracle/__init__``).

One GN iteration (Sec. 2.2, eqs. (gniter), (gniterf1), (pcgsystem); Sec. 3.2):
  1. x = x_b + Gamma^{1/2} v, forward model, innovations        (one FWD)
  2. g_v = v + A^T d                                             (one ADJ)
  3. b = -g_v
  4. optionally test a resident preconditioner with kappa_re (eq. (condtext2))
  5. otherwise sketch H (Nystrom, Alg. 2 or RandSVD, Alg. 1)    (l TLM + l ADJ)
  6. PCG on (I + H) dv = b, preconditioned by eq. (woodbury)     (one TLM+ADJ / iter)
  7. v <- v + alpha dv (alpha = 1: the paper's More-Thuente line search is an
     external toolbox; the unit GN step is the reading used here)

Counters follow Sec. 5 / Tables 2, 4: offline TLM/ADJ are those spent building
sketches; online FWD/TLM/ADJ are spent in the cost/gradient and in PCG.
"""
import numpy as np

from . import sketch as _sketch
from .pcg import pcg as _pcg


def kappa_re(prob, traj, V, lam, vhat):
    """kappa_re = ||(I + H^(k)) (I + H_hat^(k-i))^{-1} v||_2 with v a unit vector
    (eq. (condtext2); also kappa_sk of eq. (condtext) when the sketch is fresh)."""
    v = np.asarray(vhat, dtype=np.float64)
    v = v / np.linalg.norm(v)
    z = _sketch.lmp_apply(V, lam, v)
    return float(np.linalg.norm(prob.hessian(traj, z)))


def build_precond_adaptive(prob, traj, Omegas, v, eps_sk):
    """Alg. 4 on the problem's A (m x n) and H = A^T A: returns (V, lam, kappas)."""
    m = prob.m
    return _sketch.randsvd_adaptive(lambda X: prob.A(traj, X).reshape(m, -1),
                                    lambda W: prob.AT(traj, W.reshape(prob.n_t, prob.n_obs, -1)),
                                    lambda X: prob.misfit_hessian(traj, X), Omegas, v, eps_sk)


def build_precond_singleview_adaptive(prob, traj, Omegas, Psis, v, eps_sk, qr='direct'):
    """Alg. 5 on the problem's A: returns (V, lam, kappas)."""
    m = prob.m
    return _sketch.singleview_adaptive(lambda X: prob.A(traj, X).reshape(m, -1),
                                       lambda W: prob.AT(traj, W.reshape(prob.n_t, prob.n_obs, -1)),
                                       lambda X: prob.misfit_hessian(traj, X), Omegas, Psis, v, eps_sk, qr=qr)


def build_precond_nystrom_adaptive(prob, traj, Omegas, v, eps_sk):
    """Adaptive Nystrom on the problem's H: returns (V, lam, nu, kappas)."""
    return _sketch.nystrom_adaptive(lambda X: prob.misfit_hessian(traj, X), Omegas, v, eps_sk)


def split_blocks(X, first, step):
    """Columns [0, first), then `step` at a time while whole blocks remain."""
    return [X[:, :first]] + [X[:, k:k + step] for k in range(first, X.shape[1] - step + 1, step)]


def build_precond(prob, traj, method, Omega, eps=_sketch.EPS64):
    if method == 'nystrom':
        V, lam, _ = _sketch.nystrom(lambda X: prob.misfit_hessian(traj, X), Omega, eps=eps)
    elif method == 'randsvd':
        m = prob.m
        V, lam = _sketch.randsvd(lambda X: prob.A(traj, X).reshape(m, -1),
                                 lambda W: prob.AT(traj, W.reshape(prob.n_t, prob.n_obs, -1)),
                                 Omega)
    elif method == 'singleview':
        m = prob.m
        Om, Psi = Omega                                    # (n x l1, m x l2)
        V, lam = _sketch.singleview(lambda X: prob.A(traj, X).reshape(m, -1),
                                    lambda W: prob.AT(traj, W.reshape(prob.n_t, prob.n_obs, -1)), Om, Psi)
    else:
        raise ValueError(method)
    return V, lam


ARMIJO_C = 1e-4
ARMIJO_MAX_TRIALS = 20


def armijo(prob, v, J0, g, dv, counters=None):
    """Backtracking line search on the v-form cost: alpha = 1, 1/2, 1/4, ...
    until J(v + alpha dv) <= J0 + c alpha g.dv (c = 1e-4), at most 20 trials
    (the last trial's alpha is taken if none passes).  One FWD per trial.
    Returns (alpha, trials)."""
    slope = float(g @ dv)
    alpha = 1.0
    for t in range(1, ARMIJO_MAX_TRIALS + 1):
        J = prob.cost(v + alpha * dv)
        if counters is not None:
            counters['fwd'] += 1
        if J <= J0 + ARMIJO_C * alpha * slope or t == ARMIJO_MAX_TRIALS:
            return alpha, t
        alpha *= 0.5


def gn_step(prob, v, method='nystrom', Omega=None, rtol=1e-6, maxit=None,
            precond=None, reuse_eps=None, vhat=None, counters=None, adaptive=None, solve='pcg',
            line_search=False):
    """One GN step from control vector v.

    method: 'nystrom' | 'randsvd' | 'randsvd_adaptive' (Alg. 4) | 'nystrom_adaptive' | 'singleview'
    (Alg. 3; Omega is then the pair (Omega, Psi)) | 'singleview_adaptive'
    (Alg. 5; the pair again, split by adaptive['ell0'/'ell_hat'] and
    adaptive['ell2'/'ell2_hat']) | 'none' (Prec_Gamma).
    precond: optional resident (V, lam) from an earlier iterate; with reuse_eps
    set it is kept when kappa_re(vhat) < reuse_eps, otherwise rebuilt from Omega.
    adaptive: dict(ell0, ell_hat, eps_sk) for Alg. 4, whose Gaussian blocks are
    Omega's columns [0, ell0), then ell_hat at a time; vhat is its test vector.
    solve: 'pcg' (SketchPrec, Sec. 3.2.2) or 'sketch' (SketchSolv, Sec. 3.2.1:
    eq. (dxsol) in the v-form, dv = (I + H_hat)^{-1} b by eq. (woodbury)).
    line_search: take v + alpha dv with alpha from ``armijo`` instead of alpha = 1.
    Returns (v_new, dv, x_new, info)."""
    c = counters if counters is not None else dict(fwd=0, tlm_on=0, adj_on=0, tlm_off=0, adj_off=0)
    J, g, traj, x = prob.cost_grad(v)
    c['fwd'] += 1
    c['adj_on'] += 1
    b = -g
    reused = False
    kre = None
    P = None
    if method != 'none':
        if precond is not None and reuse_eps is not None:
            kre = kappa_re(prob, traj, precond[0], precond[1], vhat)
            if kre < reuse_eps:
                P = precond
                reused = True
        if P is None and method == 'randsvd_adaptive':
            blocks = split_blocks(Omega, adaptive['ell0'], adaptive['ell_hat'])
            V, lam, kappas = build_precond_adaptive(prob, traj, blocks, vhat, adaptive['eps_sk'])
            P = (V, lam)
            c['tlm_off'] += V.shape[1] + len(kappas)
            c['adj_off'] += V.shape[1] + len(kappas)
        elif P is None and method == 'nystrom_adaptive':
            blocks = split_blocks(Omega, adaptive['ell0'], adaptive['ell_hat'])
            V, lam, _, kappas = build_precond_nystrom_adaptive(prob, traj, blocks, vhat, adaptive['eps_sk'])
            P = (V, lam)
            c['tlm_off'] += V.shape[1] + len(kappas)
            c['adj_off'] += V.shape[1] + len(kappas)
        elif P is None and method == 'singleview_adaptive':
            Om, Psi = Omega
            a = adaptive
            ob = split_blocks(Om, a['ell0'], a['ell_hat'])
            pb = split_blocks(Psi, a['ell2'], a['ell2_hat'])
            V, lam, kappas = build_precond_singleview_adaptive(prob, traj, ob, pb, vhat, a['eps_sk'])
            P = (V, lam)
            r = len(kappas) - 1
            c['tlm_off'] += V.shape[1] + len(kappas)
            c['adj_off'] += a['ell2'] + r * a['ell2_hat'] + len(kappas)
        elif P is None:
            P = build_precond(prob, traj, method, Omega)
            if method == 'singleview':
                c['tlm_off'] += Omega[0].shape[1]
                c['adj_off'] += Omega[1].shape[1]
            else:
                c['tlm_off'] += Omega.shape[1]
                c['adj_off'] += Omega.shape[1]
    prec = (lambda r: _sketch.lmp_apply(P[0], P[1], r)) if P is not None else None
    if solve == 'sketch':
        if prec is None:
            raise ValueError("SketchSolv needs a sketch")
        dv, pinfo = prec(b), dict(iters=0, converged=True, relres=None)
    else:
        dv, pinfo = _pcg(lambda p: prob.hessian(traj, p), b, prec=prec, rtol=rtol, maxit=maxit)
    c['tlm_on'] += pinfo['iters']
    c['adj_on'] += pinfo['iters']
    alpha, trials = (armijo(prob, v, J, g, dv, c) if line_search else (1.0, 0))
    v_new = v + alpha * dv
    x_new = prob.state(v_new)
    info = dict(J=J, gnorm_inf=float(np.max(np.abs(g))), g=g, pcg=pinfo, reused=reused,
                kappa_re=kre, precond=P, counters=c, x=x, alpha=alpha, ls_trials=trials)
    return v_new, dv, x_new, info
