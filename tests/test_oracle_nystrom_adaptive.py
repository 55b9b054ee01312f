"""Pins of the oracle's adaptive Nystrom sketch (Sec. 3.1.2, the Nystrom form of
the adaptive loop) against facts fixed by the mathematics:
  * Nystrom approximations with nested test matrices are ordered,
    H_hat_1 <= H_hat_2 <= ... <= H (Loewner order, up to the stabilising
    shift nu), so a loop that dropped earlier blocks would fail;
  * every kappa_sk equals ||(I + H)(I + H_hat)^{-1} v|| with a dense solve;
  * a rank-r H is captured by the first block (l0 >= r): kappa_sk = 1;
  * the loop stops at the first kappa_sk <= eps_sk.
"""
import numpy as np

from oracle import sketch as osk


def _decaying_psd(n, seed, rate=0.6, scale=500.0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (U * (scale * rate ** np.arange(n))) @ U.T


def _blocks(n, seed, l0, lh, ext):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, l0))] + [rng.standard_normal((n, lh)) for _ in range(ext)]


def _hhat(V, lam):
    return (V * lam) @ V.T


def test_nested_sketches_are_loewner_ordered_and_kappa_is_the_dense_value():
    n = 40
    H = _decaying_psd(n, 1)
    Hf = lambda X: H @ X
    blocks = _blocks(n, 2, 4, 3, 4)
    v = np.random.default_rng(3).standard_normal(n)
    vu = v / np.linalg.norm(v)
    prev = np.zeros((n, n))
    for k in range(1, len(blocks) + 1):
        V, lam, nu, kap = osk.nystrom_adaptive(Hf, blocks[:k], v, eps_sk=1.0)
        assert len(kap) == k
        Hh = _hhat(V, lam)
        tol = 10 * nu * n + 1e-12 * np.linalg.norm(H, 2)
        assert np.linalg.eigvalsh(H - Hh)[0] >= -tol
        assert np.linalg.eigvalsh(Hh - prev)[0] >= -tol
        dense = np.linalg.norm((np.eye(n) + H) @ np.linalg.solve(np.eye(n) + Hh, vu))
        assert abs(kap[-1] - dense) <= 1e-10 * dense
        prev = Hh


def test_low_rank_operator_stops_at_once():
    rng = np.random.default_rng(4)
    n, r = 30, 3
    B = rng.standard_normal((n, r))
    H = B @ B.T
    V, lam, nu, kap = osk.nystrom_adaptive(lambda X: H @ X, _blocks(n, 5, 5, 2, 3), rng.standard_normal(n), 1.01)
    assert len(kap) == 1 and abs(kap[0] - 1.0) <= 1e-8
    assert np.allclose(_hhat(V, lam), H, atol=1e-8 * np.linalg.norm(H))


def test_stops_at_the_first_kappa_below_tolerance():
    n = 50
    H = _decaying_psd(n, 6, rate=0.7)
    Hf = lambda X: H @ X
    blocks = _blocks(n, 7, 3, 3, 8)
    v = np.random.default_rng(8).standard_normal(n)
    _, _, _, full = osk.nystrom_adaptive(Hf, blocks, v, eps_sk=1.0)
    eps = 0.5 * (full[2] + full[3])
    _, _, _, kap = osk.nystrom_adaptive(Hf, blocks, v, eps_sk=eps)
    assert kap[-1] <= eps and all(k > eps for k in kap[:-1])
    assert np.allclose(kap, full[:len(kap)], rtol=1e-12)


def test_gn_step_wrapper_counts():
    from oracle import gn as ogn
    from oracle.problem import burgers_problem
    from paper_2401_15758_amd import inputs
    cfg = inputs.CFG_SMALL
    orc = burgers_problem(cfg, inputs.draws(cfg, seed=0))
    Om = inputs.omega(orc.n, 16, seed=5)
    vh = inputs.omega(orc.n, 1, seed=7)[:, 0]
    c = dict(fwd=0, tlm_on=0, adj_on=0, tlm_off=0, adj_off=0)
    _, _, _, info = ogn.gn_step(orc, np.zeros(orc.n), method='nystrom_adaptive', Omega=Om, vhat=vh, rtol=1e-8,
                                counters=c, adaptive=dict(ell0=8, ell_hat=4, eps_sk=1.0))
    assert info['precond'][0].shape[1] == 16
    assert c['tlm_off'] == 16 + 3 and c['adj_off'] == 16 + 3
