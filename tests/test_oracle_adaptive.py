"""Pins of the oracle's adaptive RandSVD (Sec. 3.1.2, Alg. 4) and its test
kappa_sk (eq. (condtext)) against facts fixed by the algebra:
  * kappa_sk equals |(I + H)(I + H_hat)^{-1} v| formed from dense matrices;
  * without an extension Alg. 4 returns Alg. 1's approximation;
  * after extensions the approximation equals Alg. 1 on the concatenated
    Gaussian blocks (both are A^T Q Q^T A with Q spanning A [Omega_1 ...]);
  * kappa_sk = 1 when H_hat = H (full-rank sketch of a low-rank H).
"""
import numpy as np
import pytest

from oracle import gn as ogn
from oracle import sketch as osk
from oracle.problem import burgers_problem
from paper_2401_15758_amd import inputs

CFG = inputs.CFG_SMALL


@pytest.fixture(scope="module")
def prob():
    orc = burgers_problem(CFG, inputs.draws(CFG, seed=0))
    return orc, orc.fwd(orc.xb)


def _dense(orc, tr, fn, n):
    return fn(tr, np.eye(n))


def test_kappa_sk_matches_dense_definition():
    rng = np.random.default_rng(1)
    n, m, ell = 12, 9, 4
    A = rng.standard_normal((m, n))
    H = A.T @ A
    W = rng.standard_normal((ell, n))
    v = rng.standard_normal(n)
    direct = np.linalg.norm((np.eye(n) + H) @ np.linalg.solve(np.eye(n) + W.T @ W, v / np.linalg.norm(v)))
    assert osk.kappa_sk(lambda X: H @ X, W, v) == pytest.approx(direct, rel=1e-12)


def test_exact_sketch_gives_kappa_one():
    rng = np.random.default_rng(2)
    n, m = 10, 3
    A = rng.standard_normal((m, n))
    Om = rng.standard_normal((n, m))
    V, lam, kap = osk.randsvd_adaptive(lambda X: A @ X, lambda Y: A.T @ Y, lambda X: A.T @ (A @ X), [Om],
                                       rng.standard_normal(n), eps_sk=1.01)
    assert kap[0] == pytest.approx(1.0, abs=1e-12)
    assert np.allclose(V @ np.diag(lam) @ V.T, A.T @ A, atol=1e-11)


def test_no_extension_is_fixed_randsvd(prob):
    orc, tr = prob
    Om = inputs.omega(orc.n, 10, seed=21)
    extra = inputs.omega(orc.n, 5, seed=22)
    V, lam, kap = ogn.build_precond_adaptive(orc, tr, [Om, extra], np.ones(orc.n), eps_sk=1e30)
    assert len(kap) == 1
    V1, lam1 = ogn.build_precond(orc, tr, 'randsvd', Om)
    assert np.allclose(lam, lam1, rtol=1e-12, atol=1e-12 * lam1[0])
    X = np.random.default_rng(3).standard_normal((orc.n, 3))
    assert np.allclose(osk.hhat_apply(V, lam, X), osk.hhat_apply(V1, lam1, X), rtol=1e-10, atol=1e-10 * lam1[0])


def test_extensions_equal_randsvd_on_concatenated_blocks(prob):
    orc, tr = prob
    blocks = [inputs.omega(orc.n, 8, seed=31), inputs.omega(orc.n, 4, seed=32), inputs.omega(orc.n, 4, seed=33)]
    V, lam, kap = ogn.build_precond_adaptive(orc, tr, blocks, np.ones(orc.n), eps_sk=1.0)  # never satisfied
    assert len(kap) == 3
    assert all(k2 <= k1 * (1 + 1e-9) for k1, k2 in zip(kap, kap[1:]))   # a larger sketch never hurts here
    Vc, lamc = ogn.build_precond(orc, tr, 'randsvd', np.hstack(blocks))
    X = np.random.default_rng(4).standard_normal((orc.n, 3))
    ref = osk.hhat_apply(Vc, lamc, X)
    assert np.linalg.norm(osk.hhat_apply(V, lam, X) - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.allclose(lam[:len(lamc)], lamc, rtol=1e-9, atol=1e-10 * lamc[0])


def test_stops_at_tolerance(prob):
    orc, tr = prob
    blocks = [inputs.omega(orc.n, 8, seed=41)] + [inputs.omega(orc.n, 8, seed=42 + i) for i in range(8)]
    v = inputs.omega(orc.n, 1, seed=50)[:, 0]
    _, _, kap = ogn.build_precond_adaptive(orc, tr, blocks, v, eps_sk=1.5)
    assert kap[-1] <= 1.5 or len(kap) == len(blocks)
    assert all(k > 1.5 for k in kap[:-1])
