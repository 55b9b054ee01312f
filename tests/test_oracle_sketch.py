"""Pins of the sketch oracle: Nystrom and RandSVD against their closed-form
projector definitions (pseudo-inverse formulas of Sec. 3.1.1 / Sec. 4.4), exactness
when l >= rank, the Loewner ordering H_hat <= H (Sec. 4.3-4.4), the deterministic
condition-number bound of Thm. (bound_loew), the expectation bound of Thms.
(RandSVD)/(Nystrom), the Woodbury identities and the intrinsic-dimension closed forms."""
import numpy as np
import pytest
from scipy.special import zeta

from oracle import analysis, sketch


def _lowrank_psd(n, r, seed, decay=0.5):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    lam = 100.0 * decay ** np.arange(r)
    return (U * lam) @ U.T, U, lam


def test_nystrom_matches_pseudoinverse_formula():
    H, _, _ = _lowrank_psd(60, 30, 1, decay=0.7)
    Om = np.random.default_rng(2).standard_normal((60, 12))
    V, lam, nu = sketch.nystrom(lambda X: H @ X, Om)
    Y = H @ Om
    ref = Y @ np.linalg.pinv(Om.T @ Y) @ Y.T
    Hh = sketch.hhat_apply(V, lam, np.eye(60))
    assert np.linalg.norm(Hh - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.allclose(V.T @ V, np.eye(12), atol=1e-10)


def test_nystrom_exact_when_sketch_exceeds_rank():
    H, _, _ = _lowrank_psd(50, 6, 3)
    Om = np.random.default_rng(4).standard_normal((50, 10))
    V, lam, nu = sketch.nystrom(lambda X: H @ X, Om)
    Hh = sketch.hhat_apply(V, lam, np.eye(50))
    assert np.linalg.norm(Hh - H, 2) <= 100 * nu + 1e-12 * np.linalg.norm(H, 2)


def test_randsvd_matches_projector_formula():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 70)) * (0.6 ** np.arange(70))[None, :]
    Om = rng.standard_normal((70, 15))
    V, lam = sketch.randsvd(lambda X: A @ X, lambda W: A.T @ W, Om)
    Y = A @ Om
    P = Y @ np.linalg.pinv(Y)
    ref = A.T @ P @ A
    Hh = sketch.hhat_apply(V, lam, np.eye(70))
    assert np.linalg.norm(Hh - ref) <= 1e-11 * np.linalg.norm(ref)


def test_lmp_inverts_one_plus_hhat_and_woodbury_W_form():
    rng = np.random.default_rng(6)
    n, ell = 80, 10
    V, _ = np.linalg.qr(rng.standard_normal((n, ell)))
    lam = np.abs(rng.standard_normal(ell)) * 10
    lam[-1] = 0.0
    M = np.eye(n) + (V * lam) @ V.T
    P = sketch.lmp_apply(V, lam, np.eye(n))
    assert np.linalg.norm(P @ M - np.eye(n)) <= 1e-13 * n
    W = rng.standard_normal((ell, n))
    r = rng.standard_normal(n)
    ref = np.linalg.solve(np.eye(n) + W.T @ W, r)
    assert np.allclose(sketch.woodbury_W_apply(W, r), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("method", ["nystrom", "randsvd"])
def test_loewner_order_and_condition_bound_on_burgers(small_problem, small_dense, method):
    """Thm. (bound_loew) special case: E = H - H_hat >= 0 and
    kappa_2 <= 1 + ||E||_2 for every seed and sketch size (deterministic)."""
    p = small_problem
    traj, Hs, _ = small_dense
    A = None
    if method == 'randsvd':
        A = p.A(traj, np.eye(p.n)).reshape(p.m, p.n)
    for ell in (5, 10, 20, 40):
        for seed in range(4):
            Om = np.random.default_rng(1000 + seed).standard_normal((p.n, ell))
            if method == 'nystrom':
                V, lam, nu = sketch.nystrom(lambda X: Hs @ X, Om)
            else:
                V, lam = sketch.randsvd(lambda X: A @ X, lambda W: A.T @ W, Om)
                nu = 0.0
            Hh = sketch.hhat_apply(V, lam, np.eye(p.n))
            E = Hs - 0.5 * (Hh + Hh.T)
            wE = np.linalg.eigvalsh(E)
            tol = 1e-13 * np.linalg.norm(Hs, 2) + 10 * nu
            assert wE[0] >= -tol
            kap = analysis.precond_kappa(Hs, Hh)
            assert kap <= 1 + wE[-1] + 1e-8 * (1 + wE[-1])


@pytest.mark.parametrize("method", ["nystrom", "randsvd"])
def test_expected_condition_bound(small_problem, small_dense, method):
    """Thms. (RandSVD), (Nystrom): E[kappa_2] <= 1 + Psi_H(r, p), checked with the
    sample mean over 40 seeds (the bound holds with margin for this spectrum)."""
    p = small_problem
    traj, Hs, _ = small_dense
    lamH = np.linalg.eigvalsh(Hs)[::-1]
    ell, r = 20, 14
    A = p.A(traj, np.eye(p.n)).reshape(p.m, p.n) if method == 'randsvd' else None
    kaps = []
    for seed in range(40):
        Om = np.random.default_rng(5000 + seed).standard_normal((p.n, ell))
        if method == 'nystrom':
            V, lam, _ = sketch.nystrom(lambda X: Hs @ X, Om)
        else:
            V, lam = sketch.randsvd(lambda X: A @ X, lambda W: A.T @ W, Om)
        kaps.append(analysis.precond_kappa(Hs, sketch.hhat_apply(V, lam, np.eye(p.n))))
    bound = 1 + analysis.psi_bound(lamH, r, ell - r)
    assert np.mean(kaps) <= bound, (np.mean(kaps), bound)


def test_intrinsic_dimension_closed_forms():
    """Sec. 4.2: for lambda_j = j^-alpha the tail ratio is (r+1)^alpha zeta(alpha, r+1)
    (Hurwitz zeta), which equals the paper's zeta(alpha) bound at r = 0 and exceeds it
    for r > 0 (the printed bound holds only for the untruncated spectrum); for
    lambda_j = exp(-alpha j) it is exactly 1/(1 - exp(-alpha)) for an infinite tail."""
    j = np.arange(1, 200001, dtype=np.float64)
    for alpha in (2.0, 3.0, 4.0):
        lam = j ** (-alpha)
        assert analysis.intrinsic_dimension(lam, 0) <= zeta(alpha) + 1e-12
        for r in (0, 3, 10):
            ref = (r + 1) ** alpha * zeta(alpha, r + 1)
            assert analysis.intrinsic_dimension(lam, r) == pytest.approx(ref, rel=1e-3)
    for alpha in (0.1, 0.5, 2.0):
        lam = np.exp(-alpha * np.arange(1, 4000))
        idr = analysis.intrinsic_dimension(lam, 5)
        assert idr <= 1 / (1 - np.exp(-alpha)) + 1e-12
        assert idr == pytest.approx(1 / (1 - np.exp(-alpha)), rel=1e-9)


def test_sample_size_rule():
    """Sec. 4.2 'Number of samples': l = ceil(6 r_eps/5 + 1) gives Psi <= (1 + 5 id) eps."""
    lam = 10.0 * 0.7 ** np.arange(200)
    for eps in (1e-1, 1e-2, 1e-3):
        r_eps = int(np.sum(lam > eps))
        ell = int(np.ceil(6 * r_eps / 5 + 1))
        p = ell - r_eps
        if p < 2:
            continue
        psi = analysis.psi_bound(lam, r_eps, p)
        assert psi <= (1 + 5 * analysis.intrinsic_dimension(lam, r_eps)) * eps


def test_singleview_expected_bounds(small_problem, small_dense):
    """Thm. (SingleView) with l1 = 2r + 1, l2 = 2 l1 + 1: the sample means over
    30 seeds of sqrt(kappa_2) and of the SketchSolv error |dv - dv_hat|/|dv|
    (eq. (dxsol), the Gamma^{-1} norm of the x-step) stay within 1 + Theta_H(r)
    and Theta_H(r).  SingleView's H - H_hat is not PSD in general, so each draw
    also obeys the weaker deterministic bound sqrt(kappa_2) <= 1 + |E|_2 of
    Thm. (bound_loew)."""
    p = small_problem
    traj, Hs, _ = small_dense
    lamH = np.linalg.eigvalsh(Hs)[::-1]
    A = p.A(traj, np.eye(p.n)).reshape(p.m, p.n)
    r = 6
    l1, l2 = 2 * r + 1, 2 * (2 * r + 1) + 1
    b = np.random.default_rng(77).standard_normal(p.n)
    dv = np.linalg.solve(np.eye(p.n) + Hs, b)
    roots, errs = [], []
    for seed in range(30):
        rng = np.random.default_rng(6000 + seed)
        V, lam = sketch.singleview(lambda X: A @ X, lambda W: A.T @ W, rng.standard_normal((p.n, l1)),
                                   rng.standard_normal((p.m, l2)))
        Hh = sketch.hhat_apply(V, lam, np.eye(p.n))
        kap = analysis.precond_kappa(Hs, Hh)
        E = np.linalg.norm(Hs - Hh, 2)
        assert np.sqrt(kap) <= 1 + E + 1e-8 * (1 + E)
        roots.append(np.sqrt(kap))
        errs.append(np.linalg.norm(dv - sketch.lmp_apply(V, lam, b)) / np.linalg.norm(dv))
    theta = analysis.theta_bound(lamH, r)
    assert np.mean(roots) <= 1 + theta, (np.mean(roots), theta)
    assert np.mean(errs) <= theta, (np.mean(errs), theta)


# --- the Nystrom shift and its retries (Alg. 2; reading: x10 per retry, at most 3) ---

def _indefinite_sketch(n, delta, ratio, seed):
    """A square Gaussian Omega (n x n, invertible) and Y0 = H Omega for a
    symmetric H with one eigenvalue -delta and the others positive, scaled so
    that the first shift nu0 = sqrt(n) eps ||Y0||_2 equals delta / ratio."""
    rng = np.random.default_rng(seed)
    Om = rng.standard_normal((n, n))
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.linspace(1.0, 2.0, n)
    lam[-1] = 0.0
    # the positive part sets ||Y0||_2; choose its scale c so that nu0 = delta / ratio
    base = np.linalg.norm((U * lam) @ U.T @ Om, 2)
    c = delta / ratio / (np.sqrt(n) * sketch.EPS64 * base)
    lam = c * lam
    lam[-1] = -delta
    H = (U * lam) @ U.T
    return Om, H @ Om, H, lam


@pytest.mark.parametrize("ratio, retries", [(3.0, 1), (30.0, 2), (300.0, 3)])
def test_nystrom_shift_retries(ratio, retries):
    """With H + nu I indefinite at the first shift (one eigenvalue -delta, and
    nu0 = delta / ratio), the core Omega^T (H + nu I) Omega of a square,
    invertible Omega is positive definite exactly when nu > delta: the shift
    must be retried `retries` times, ending at nu = 10^retries nu0.  For a
    square Omega the Nystrom approximant of H + nu I is H + nu I itself, so the
    returned eigenvalues are max(0, eig(H))."""
    n, delta = 12, 1e-3
    Om, Y0, H, lam = _indefinite_sketch(n, delta, ratio, seed=11)
    nu0 = np.sqrt(n) * sketch.EPS64 * np.linalg.norm(Y0, 2)
    assert nu0 == pytest.approx(delta / ratio, rel=1e-12)
    V, lh, nu = sketch.nystrom_from_sketch(Om, Y0)
    assert nu == pytest.approx(10.0 ** retries * nu0, rel=1e-14)
    ref = np.sort(np.maximum(0.0, lam))[::-1]
    got = np.sort(lh)[::-1]
    # the clamped direction keeps an error of order nu (its shifted eigenvalue
    # nu - delta > 0 loses nu); the rest are exact up to cond(Omega) eps |H|
    assert np.max(np.abs(got - ref)) <= 1e-8 * ref[0]


def test_nystrom_shift_gives_up_after_three_retries():
    n, delta = 12, 1e-3
    Om, Y0, _, _ = _indefinite_sketch(n, delta, 3000.0, seed=12)   # 1000 nu0 < delta
    with pytest.raises(sketch.NotSPDError):
        sketch.nystrom_from_sketch(Om, Y0)
    # with more retries allowed the fourth one (10^4 nu0 > delta) succeeds
    _, _, nu = sketch.nystrom_from_sketch(Om, Y0, max_retries=4)
    assert nu == pytest.approx(1e4 * np.sqrt(n) * sketch.EPS64 * np.linalg.norm(Y0, 2), rel=1e-14)


def test_nystrom_zero_column_is_never_positive_definite():
    """A zero column of Omega gives a zero row and column of the core at every
    shift: every retry fails."""
    rng = np.random.default_rng(13)
    A = rng.standard_normal((30, 40))
    Om = rng.standard_normal((40, 8))
    Om[:, 5] = 0.0
    with pytest.raises(sketch.NotSPDError):
        sketch.nystrom(lambda X: A.T @ (A @ X), Om)


# --- Sec. 4 bounds, exact values on a closed-form spectrum ---

def test_psi_and_theta_exact_on_a_geometric_spectrum():
    """lambda_j = 2^{-(j-1)}, j = 1..10.  The tail sums are geometric:
    sum_{j>r} lambda_j = 2^{-r} (2 - 2^{-(9-r)}) ... written out for r = 2:
    lambda_3 = 1/4, sum_{j>2} lambda_j = 1/4 (1 + 1/2 + ... + 1/128) = 255/512.
    Psi_H(r, p) = lambda_{r+1} + r/(p-1) sum_{j>r} lambda_j (the first form of
    the definition), with r = 2, p = 3: 1/4 + 255/512 = 383/512.
    Theta_H(r) in its second form, (sqrt(lambda_1/lambda_{r+1}) sqrt(id_r) + id_r)
    4 lambda_{r+1} with id_r = (255/512)/(1/4) = 255/128: (2 sqrt(255/128) +
    255/128)."""
    lam = 2.0 ** -np.arange(10)
    rng = np.random.default_rng(0)
    shuffled = rng.permutation(lam)                  # the functions sort themselves
    assert analysis.intrinsic_dimension(shuffled, 2) == 255.0 / 128.0
    assert analysis.psi_bound(shuffled, 2, 3) == 383.0 / 512.0
    # the second form of the definition, (1 + r/(p-1) id_r) lambda_{r+1}, agrees
    assert (1.0 + 255.0 / 128.0) / 4.0 == 383.0 / 512.0
    idr = 255.0 / 128.0
    assert analysis.theta_bound(shuffled, 2) == pytest.approx((2.0 * np.sqrt(idr) + idr), rel=1e-15)
    # r = 0: Psi = lambda_1 + 0 = 1, Theta = 4 sqrt(sum) + 4 sum with sum = 1023/512
    s0 = 1023.0 / 512.0
    assert analysis.psi_bound(lam, 0, 2) == 1.0
    assert analysis.theta_bound(lam, 0) == pytest.approx(4.0 * np.sqrt(s0) + 4.0 * s0, rel=1e-15)
    # a flat spectrum of rank 5: Psi vanishes once r reaches the rank
    flat = np.r_[np.ones(5), np.zeros(5)]
    assert analysis.psi_bound(flat, 5, 3) == 0.0 and analysis.theta_bound(flat, 5) == 0.0
    assert analysis.psi_bound(flat, 4, 3) == 1.0 + 4.0 / 2.0 * 1.0
