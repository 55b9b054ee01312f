"""Pins of the oracle's adaptive SingleView (Sec. 3.1.2, Alg. 5) and its QR
update (Alg. 6) against facts fixed by the algebra:
  * Alg. 6 returns a thin QR of the stacked product: Q5 R5 reproduces it, Q5 has
    orthonormal columns and R5 is upper triangular, and |diag R5| matches a
    direct Householder QR (the thin QR of a full-rank matrix is unique up to
    signs);
  * the SingleView approximation depends only on range(Y), Psi and Z, so after
    any number of extensions the adaptive result equals Alg. 3 on the
    concatenated test matrices, and every kappa_sk equals eq. (condtext) for
    Alg. 3 on the blocks drawn so far;
  * updating M's QR by Alg. 6 or refactoring it gives the same sketch;
  * for A of rank <= l1 the first sketch is exact and kappa_sk = 1.
"""
import numpy as np

from oracle import sketch as osk


def _ops(A):
    return (lambda X: A @ X), (lambda Y: A.T @ Y), (lambda X: A.T @ (A @ X))


def _decaying(m, n, seed, rate=0.7):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, min(m, n))))
    V, _ = np.linalg.qr(rng.standard_normal((n, min(m, n))))
    s = 30.0 * rate ** np.arange(min(m, n))
    return U @ np.diag(s) @ V.T


def test_qr_update_is_a_thin_qr():
    rng = np.random.default_rng(1)
    m, c, ch, r1, r2 = 40, 6, 4, 13, 5      # A2 B1 is 5 x 6: wider than tall
    B, _ = np.linalg.qr(rng.standard_normal((m, c + ch)))
    B1, B2 = B[:, :c], B[:, c:]
    A1, A2 = rng.standard_normal((r1, m)), rng.standard_normal((r2, m))
    Q1, R1 = np.linalg.qr(A1 @ B1)
    Q5, R5 = osk.qr_update(A1, A2, B1, B2, Q1, R1)
    full = np.vstack([A1, A2]) @ B
    assert np.allclose(Q5 @ R5, full, atol=1e-12 * np.linalg.norm(full))
    assert np.allclose(Q5.T @ Q5, np.eye(c + ch), atol=1e-12)
    assert np.allclose(np.tril(R5, -1), 0.0)
    _, R = np.linalg.qr(full)
    assert np.allclose(np.abs(np.diag(R5)), np.abs(np.diag(R)), rtol=1e-10)


def _blocks(n, m, seed, l1, l2, l1h, l2h, ext):
    rng = np.random.default_rng(seed)
    Oms = [rng.standard_normal((n, l1))] + [rng.standard_normal((n, l1h)) for _ in range(ext)]
    Psis = [rng.standard_normal((m, l2))] + [rng.standard_normal((m, l2h)) for _ in range(ext)]
    return Oms, Psis


def _hhat(V, lam):
    return V @ np.diag(lam) @ V.T


def test_adaptive_equals_one_shot_on_concatenated_blocks():
    m, n = 50, 70
    A = _decaying(m, n, 2)
    Af, ATf, Hf = _ops(A)
    Oms, Psis = _blocks(n, m, 3, 5, 11, 3, 6, 3)
    v = np.random.default_rng(4).standard_normal(n)
    V, lam, kap = osk.singleview_adaptive(Af, ATf, Hf, Oms, Psis, v, eps_sk=1.0 + 1e-14)
    assert len(kap) == 4                    # never met: every block is used
    Vo, lo = osk.singleview(Af, ATf, np.hstack(Oms), np.hstack(Psis))
    H0 = _hhat(Vo, lo)
    assert np.allclose(_hhat(V, lam), H0, atol=1e-10 * np.linalg.norm(H0))
    for j in range(4):
        Vj, lj = osk.singleview(Af, ATf, np.hstack(Oms[:j + 1]), np.hstack(Psis[:j + 1]))
        Wj = np.sqrt(lj)[:, None] * Vj.T    # H_hat = W^T W
        assert abs(kap[j] - osk.kappa_sk(Hf, Wj, v)) <= 1e-10 * kap[j]


def test_qr_update_and_direct_refactorisation_agree():
    m, n = 60, 45
    A = _decaying(m, n, 5, rate=0.8)
    Af, ATf, Hf = _ops(A)
    Oms, Psis = _blocks(n, m, 6, 4, 9, 4, 8, 2)
    v = np.random.default_rng(7).standard_normal(n)
    a = osk.singleview_adaptive(Af, ATf, Hf, Oms, Psis, v, eps_sk=1.0, qr='direct')
    b = osk.singleview_adaptive(Af, ATf, Hf, Oms, Psis, v, eps_sk=1.0, qr='update')
    assert np.allclose(a[2], b[2], rtol=1e-10)
    Ha = _hhat(a[0], a[1])
    assert np.allclose(_hhat(b[0], b[1]), Ha, atol=1e-10 * np.linalg.norm(Ha))


def test_low_rank_is_exact_at_once_and_stops():
    rng = np.random.default_rng(8)
    m, n, r = 30, 40, 4
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    Af, ATf, Hf = _ops(A)
    Oms, Psis = _blocks(n, m, 9, 6, 13, 3, 6, 2)
    V, lam, kap = osk.singleview_adaptive(Af, ATf, Hf, Oms, Psis, rng.standard_normal(n), eps_sk=1.01)
    assert len(kap) == 1 and abs(kap[0] - 1.0) <= 1e-9
    assert np.allclose(_hhat(V, lam), A.T @ A, atol=1e-9 * np.linalg.norm(A) ** 2)


def test_stops_at_the_first_kappa_below_tolerance():
    m, n = 50, 70
    A = _decaying(m, n, 10, rate=0.6)
    Af, ATf, Hf = _ops(A)
    Oms, Psis = _blocks(n, m, 11, 3, 7, 3, 6, 5)
    v = np.random.default_rng(12).standard_normal(n)
    _, _, full = osk.singleview_adaptive(Af, ATf, Hf, Oms, Psis, v, eps_sk=1.0)
    eps = 0.5 * (full[1] + full[2]) if full[2] < full[1] else full[2] * 1.000001
    _, _, kap = osk.singleview_adaptive(Af, ATf, Hf, Oms, Psis, v, eps_sk=eps)
    assert kap[-1] <= eps and all(k > eps for k in kap[:-1])
    assert np.allclose(kap, full[:len(kap)], rtol=1e-12)


def test_gn_step_wrapper_counts_blocks():
    from oracle import gn as ogn
    from oracle.problem import burgers_problem
    from paper_2401_15758_amd import inputs
    cfg = inputs.CFG_SMALL
    orc = burgers_problem(cfg, inputs.draws(cfg, seed=0))
    Om = inputs.omega(orc.n, 16, seed=5)
    Psi = np.random.default_rng(6).standard_normal((orc.m, 33))
    vh = inputs.omega(orc.n, 1, seed=7)[:, 0]
    c = dict(fwd=0, tlm_on=0, adj_on=0, tlm_off=0, adj_off=0)
    _, _, _, info = ogn.gn_step(orc, np.zeros(orc.n), method='singleview_adaptive', Omega=(Om, Psi), vhat=vh,
                                rtol=1e-8, counters=c,
                                adaptive=dict(ell0=8, ell_hat=4, ell2=17, ell2_hat=8, eps_sk=1.0))
    V = info['precond'][0]
    assert V.shape[1] == 16                          # 8 + 4 + 4: every block used
    assert c['tlm_off'] == 16 + 3 and c['adj_off'] == 33 + 3
