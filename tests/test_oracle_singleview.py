"""Pins of the oracle's SingleView approximation (Sec. 3.1.1, Alg. 3) against
facts fixed by the algebra:
  * with Psi = I (l2 = m) the oblique projector Q_Y (Psi^T Q_Y)^+ Psi^T is the
    orthogonal projector Q_Y Q_Y^T, so Alg. 3 returns Alg. 1's approximation;
  * it is exact when A has rank <= l1;
  * it equals A_SV^T A_SV with A_SV = Q_Y (Psi^T Q_Y)^+ Z^T of eq.
    (singleviewlr), formed with a dense pseudo-inverse.
"""
import numpy as np

from oracle import gn as ogn
from oracle import sketch as osk
from oracle.problem import burgers_problem
from paper_2401_15758_amd import inputs


def _ops(A):
    return (lambda X: A @ X), (lambda Y: A.T @ Y)


def test_identity_psi_reproduces_randsvd():
    rng = np.random.default_rng(1)
    m, n, l1 = 9, 14, 5
    A = rng.standard_normal((m, n))
    Om = rng.standard_normal((n, l1))
    V, lam = osk.singleview(*_ops(A), Om, np.eye(m))
    V1, lam1 = osk.randsvd(*_ops(A), Om)
    assert np.allclose(lam, lam1, rtol=1e-12)
    assert np.allclose(V @ np.diag(lam) @ V.T, V1 @ np.diag(lam1) @ V1.T, atol=1e-12 * lam1[0])


def test_exact_for_low_rank_operator():
    rng = np.random.default_rng(2)
    m, n, r = 12, 20, 3
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    V, lam = osk.singleview(*_ops(A), rng.standard_normal((n, 4)), rng.standard_normal((m, 9)))
    assert np.allclose(V @ np.diag(lam) @ V.T, A.T @ A, atol=1e-10 * np.linalg.norm(A) ** 2)


def test_matches_pseudoinverse_form():
    rng = np.random.default_rng(3)
    m, n, l1, l2 = 15, 25, 6, 13
    A = rng.standard_normal((m, n))
    Om, Psi = rng.standard_normal((n, l1)), rng.standard_normal((m, l2))
    V, lam = osk.singleview(*_ops(A), Om, Psi)
    Qy, _ = np.linalg.qr(A @ Om)
    Asv = Qy @ np.linalg.pinv(Psi.T @ Qy) @ (A.T @ Psi).T
    assert np.allclose(V @ np.diag(lam) @ V.T, Asv.T @ Asv, atol=1e-10 * np.linalg.norm(Asv) ** 2)


def test_problem_wrapper_runs():
    cfg = inputs.CFG_SMALL
    orc = burgers_problem(cfg, inputs.draws(cfg, seed=0))
    tr = orc.fwd(orc.xb)
    Om = inputs.omega(orc.n, 10, seed=5)
    Psi = np.random.default_rng(6).standard_normal((orc.m, 21))
    V, lam = ogn.build_precond(orc, tr, 'singleview', (Om, Psi))
    assert V.shape == (orc.n, 10) and np.all(lam >= 0) and np.all(np.diff(lam) <= 1e-9 * lam[0])


def test_gn_step_counts_both_sketches():
    cfg = inputs.CFG_SMALL
    orc = burgers_problem(cfg, inputs.draws(cfg, seed=0))
    Om = inputs.omega(orc.n, 6, seed=5)
    Psi = np.random.default_rng(6).standard_normal((orc.m, 13))
    c = dict(fwd=0, tlm_on=0, adj_on=0, tlm_off=0, adj_off=0)
    v1, dv, x1, info = ogn.gn_step(orc, np.zeros(orc.n), method='singleview', Omega=(Om, Psi), rtol=1e-8,
                                   counters=c)
    assert c['tlm_off'] == 6 and c['adj_off'] == 13
    assert info['pcg']['converged']
