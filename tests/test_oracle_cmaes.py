"""Pins of the CMA-ES oracle (Sec. III-A.1, Eq. cmaes_update; Sec. III-B
block-diagonal covariance; Sec. IV Sigma^(0) = I).

* Philox4x32-10 against the published known-answer vectors of its authors
  (Salmon et al., SC'11, Random123 distribution).
* Box-Muller output moments.
* Convergence on the sphere, ranking-only invariance (the paper: the update
  depends only on the fitness ranking), sigma growth on a linear function,
  symmetric positive-definite C, block-diagonal zeros.
* The mean and covariance update equal the paper's Eq. cmaes_update written in
  the paper's own variables (Theta_i, mu, sigma_k) whenever h_sigma = 1.
"""
import math

import numpy as np
import pytest

from oracle import cmaes

KAT = [  # counter (4 words), key (2 words) -> output (4 words)
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff, 0xffffffff), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_known_answers(ctr, key, out):
    got = cmaes.philox4x32_10(np.array(ctr, dtype=np.uint64), key)
    assert tuple(int(x) for x in got) == out


def test_box_muller_moments():
    z = cmaes.normals(seed=77, gen=0, lam=20000, n=9)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.02
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(9)).max() < 0.03
    # independent generations and seeds give different draws
    assert not np.array_equal(cmaes.normals(77, 1, 4, 9), cmaes.normals(77, 0, 4, 9))
    assert not np.array_equal(cmaes.normals(78, 0, 4, 9), cmaes.normals(77, 0, 4, 9))


def _run(fun, n=9, lam=16, gens=200, seed=1, m0=3.0, sigma0=1.0, n_blocks=1, **kw):
    es = cmaes.CMAES(n, lam, np.full(n, m0), sigma0, np.zeros(n), np.ones(n), seed, n_blocks=n_blocks, **kw)
    hist = []
    for _ in range(gens):
        X = es.sample()
        es.update(fun(X))
        hist.append((es.m.copy(), es.sigma, es.C.copy()))
    return es, hist


def sphere(X):
    return np.sum(X ** 2, axis=1)


def test_constants():
    k = cmaes.default_constants(9, 16)
    assert k["mu"] == 8
    assert np.sum(k["weights"]) == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.diff(k["weights"]) < 0) and np.all(k["weights"] > 0)
    # mu_eff depends only on lambda
    assert k["mu_eff"] == pytest.approx(4.8409, abs=1e-4)
    assert cmaes.default_constants(3, 70)["mu_eff"] == pytest.approx(19.187, abs=1e-3)
    assert cmaes.default_constants(18, 256)["mu_eff"] == pytest.approx(66.858, abs=1e-3)
    assert 0 < k["c1"] + k["c_mu"] <= 1
    assert 0 < k["c_sigma"] < 1 and k["d_sigma"] >= 1


GENS_SPHERE = 180   # measured on this oracle: seeds 0-19 reach 1e-10 in 122-139 generations


def test_sphere_converges_for_20_seeds():
    worst = 0
    for seed in range(20):
        es = cmaes.CMAES(9, 16, np.full(9, 3.0), 1.0, np.zeros(9), np.ones(9), seed)
        for g in range(GENS_SPHERE):
            es.update(sphere(es.sample()))
            if float(np.sum(es.m ** 2)) <= 1e-10:
                worst = max(worst, g + 1)
                break
        else:
            pytest.fail(f"seed {seed} did not reach 1e-10 in {GENS_SPHERE} generations")
    assert worst < GENS_SPHERE


def test_ranking_invariance_bit_identical():
    """Strictly increasing transforms of the loss leave the trajectory
    bit-identical: the update uses the ranking only."""
    _, h1 = _run(sphere, gens=40)
    _, h2 = _run(lambda X: np.exp(np.sqrt(sphere(X))) * 5 + 1, gens=40)
    for (m1, s1, C1), (m2, s2, C2) in zip(h1, h2):
        assert np.array_equal(m1, m2) and s1 == s2 and np.array_equal(C1, C2)


def test_ties_broken_by_index_and_nan_last():
    loss = np.array([2.0, 1.0, np.nan, 1.0, 0.5, 2.0])
    assert list(cmaes.CMAES.ranking(loss)) == [4, 1, 3, 0, 5, 2]


def test_linear_function_sigma_grows():
    es, hist = _run(lambda X: X[:, 0], gens=30, m0=0.0)
    sig = np.array([h[1] for h in hist])
    assert sig[-1] > 20 * sig[0]
    assert np.all(np.diff(np.log(sig[5:])) > 0)


def test_covariance_stays_symmetric_pd():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(9, 9))
    H = A @ A.T + np.eye(9)
    es, hist = _run(lambda X: np.einsum("ki,ij,kj->k", X, H, X), gens=120, lam=20)
    for _, _, C in hist:
        assert np.array_equal(C, C.T)
        assert np.linalg.eigvalsh(C).min() > 0
    np.testing.assert_allclose(es.L @ es.L.T, es.C, atol=1e-13 * np.abs(es.C).max())
    es._decompose()
    np.testing.assert_allclose(es.B @ np.diag(es.D ** 2) @ es.B.T, es.C, atol=1e-12 * np.abs(es.C).max())
    np.testing.assert_allclose(es.B.T @ es.B, np.eye(9), atol=1e-13)


def test_block_diagonal_keeps_zero_blocks():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(18, 18))
    H = A @ A.T + np.eye(18)            # strongly coupled objective
    es, hist = _run(lambda X: np.einsum("ki,ij,kj->k", X, H, X), n=18, lam=32, gens=60, n_blocks=2)
    for _, _, C in hist:
        assert np.all(C[:9, 9:] == 0.0) and np.all(C[9:, :9] == 0.0)
    assert np.all(es.B[:9, 9:] == 0.0) and np.all(es.B[9:, :9] == 0.0)
    assert np.all(es.L[:9, 9:] == 0.0) and np.all(es.L[9:, :9] == 0.0)


# ---------------------------------------------------------------- sampling square root
#
# y = L z with L L^T = C: the oracle's recurrences against numpy's Cholesky
# (a library routine), per block, and the pivot floor on a singular matrix.

@pytest.mark.parametrize("n,nb", [(9, 1), (18, 2), (18, 1), (3, 1)])
def test_cholesky_matches_library_routine(n, nb):
    rng = np.random.default_rng(n + nb)
    C = np.zeros((n, n))
    s = n // nb
    for b in range(nb):
        A = rng.normal(size=(s, s))
        C[b * s:(b + 1) * s, b * s:(b + 1) * s] = A @ A.T + 0.1 * np.eye(s)
    L, floored = cmaes.cholesky_floored(C, nb)
    assert not floored
    assert np.all(np.triu(L, 1) == 0.0) and np.all(np.diag(L) > 0)
    for b in range(nb):
        blk = slice(b * s, (b + 1) * s)
        np.testing.assert_allclose(L[blk, blk], np.linalg.cholesky(C[blk, blk]), rtol=0, atol=1e-13)
    if nb > 1:
        assert np.all(L[:s, s:] == 0.0) and np.all(L[s:, :s] == 0.0)


def test_cholesky_floors_a_singular_pivot():
    """C = [[1, 1, 0], [1, 1, 0], [0, 0, 4]] is positive semi-definite with an
    exactly zero second pivot: it becomes the floor 1e-20 max C_ii, the flag is
    set and L L^T = C + floor e_1 e_1^T."""
    C = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 4.0]])
    L, floored = cmaes.cholesky_floored(C)
    floor = 1e-20 * 4.0
    assert floored
    assert L[1, 1] == math.sqrt(floor) and L[2, 2] == 2.0
    E = np.zeros((3, 3))
    E[1, 1] = floor
    np.testing.assert_allclose(L @ L.T, C + E, rtol=0, atol=1e-15)
    # a positive definite matrix is not floored
    assert not cmaes.cholesky_floored(C + 1e-3 * np.eye(3))[1]


def test_samples_have_covariance_C():
    """y = L z over many draws has sample covariance C (5 standard errors)."""
    _, _, C = _fixed_state(9, 5)
    es = cmaes.CMAES(9, 20000, np.zeros(9), 1.0, np.zeros(9), np.ones(9), seed=8)
    es.set_covariance(C)
    es.sample()
    cov = np.cov(es.Y.T)
    assert np.all(np.abs(cov - C) <= _cov_bound(C, 20000))


def test_update_matches_paper_equation_in_theta_form():
    """With h_sigma = 1 the update is the paper's Eq. cmaes_update written in
    terms of the sampled states Theta_i, the old mean mu and sigma_k."""
    n, lam = 9, 16
    rng = np.random.default_rng(9)
    A = rng.normal(size=(n, n))
    H = A @ A.T + np.eye(n)
    f = lambda X: np.einsum("ki,ij,kj->k", X, H, X)
    es = cmaes.CMAES(n, lam, rng.normal(size=n), 0.7, np.zeros(n), np.ones(n), 5)
    checked = 0
    for g in range(6):
        mu_old, sig_old, C_old = es.m.copy(), es.sigma, es.C.copy()
        Theta = es.sample()                   # offset 0, scale 1: Theta = x
        loss = f(Theta)
        order = np.lexsort((np.arange(lam), loss))
        es.update(loss)
        if es.h_sigma != 1.0:
            continue
        k = es.k
        w = k["weights"]
        elite = Theta[order[:k["mu"]]]
        mu_new = mu_old + k["c_m"] * np.sum(w[:, None] * (elite - mu_old), 0)
        d = (elite - mu_old) / sig_old
        Sigma = (1 - k["c1"] - k["c_mu"]) * C_old + k["c1"] * np.outer(es.p_c, es.p_c) \
            + k["c_mu"] * np.einsum("i,ij,ik->jk", w, d, d)
        np.testing.assert_allclose(es.m, mu_new, rtol=0, atol=1e-13)
        np.testing.assert_allclose(es.C, 0.5 * (Sigma + Sigma.T), rtol=0, atol=1e-13)
        checked += 1
    assert checked >= 3


# ---------------------------------------------------------------- random selection
#
# Under selection that ignores the candidates (the loss a seeded random
# permutation, drawn independently of the samples), the update of Eq. (3)-(4)
# with Hansen's step-size and path rules must be unbiased: the tutorial builds
# every rule so that, without selection pressure, E[m'] = m, E[C'] = C, the
# conjugate path p_sigma keeps the distribution N(0, I) whatever C is, and
# E[ln sigma'] = ln sigma.  These facts follow from the mathematics alone
# (y_i:lambda are then i.i.d. N(0, C), z_i:lambda i.i.d. N(0, I)), so they pin
# the sampling square root, the weights, C^(-1/2) in the path, the path
# normalisations and the covariance learning rates without restating them.
# A non-isotropic C (eigenvalues 1 .. 100, rotated) makes a C^(+1/2) for
# C^(-1/2) slip, a missing sqrt(mu_eff) or a wrong weight sum visible.

N_TRIALS = 3000


def _fixed_state(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.linspace(1.0, 100.0, n)
    return Q, ev, Q @ np.diag(ev) @ Q.T


def _random_selection_trials(n, lam, p_sigma_stationary, p_c_stationary, seed=123):
    Q, ev, C = _fixed_state(n, seed)
    Lc = np.linalg.cholesky(C)
    rng = np.random.default_rng(seed + 1)
    m0 = rng.normal(size=n)
    sigma0 = 0.3
    out = {"dm": [], "ps": [], "C": [], "dlogs": []}
    for t in range(N_TRIALS):
        es = cmaes.CMAES(n, lam, m0, sigma0, np.zeros(n), np.ones(n), seed=1000 + t)
        es.set_covariance(C)
        es.g = 1000                          # h_sigma's start-up correction has died out
        es.p_sigma = rng.normal(size=n) if p_sigma_stationary else np.zeros(n)
        es.p_c = Lc @ rng.normal(size=n) if p_c_stationary else np.zeros(n)
        es.sample()
        es.update(rng.permutation(lam).astype(np.float64))   # selection blind to the samples
        out["dm"].append((es.m - m0) / (es.k["c_m"] * sigma0))
        out["ps"].append(es.p_sigma.copy())
        out["C"].append(es.C.copy())
        out["dlogs"].append(math.log(es.sigma / sigma0))
    return {k: np.array(v) for k, v in out.items()}, C, es.k


def _cov_bound(S, N):
    """5 standard errors of the sample covariance of N Gaussian draws with covariance S."""
    d = np.sqrt(np.diag(S))
    return 5.0 * np.sqrt((np.outer(d, d) ** 2 + S ** 2) / N)


@pytest.mark.parametrize("lam", [16, 70])
def test_random_selection_mean_step_has_covariance_C_over_mu_eff(lam):
    """m' - m = c_m sigma y_w with y_w ~ N(0, C / mu_eff): zero mean and
    mu_eff * Cov = C (pins y = L z and the normalised weights)."""
    n = 9
    r, C, k = _random_selection_trials(n, lam, False, False)
    dm = r["dm"]
    se = np.sqrt(np.diag(C) / k["mu_eff"] / N_TRIALS)
    assert np.all(np.abs(dm.mean(0)) <= 5.0 * se)
    cov = k["mu_eff"] * np.cov(dm.T)
    assert np.all(np.abs(cov - C) <= _cov_bound(C, N_TRIALS))


@pytest.mark.parametrize("lam", [16, 70])
def test_random_selection_conjugate_path_is_isotropic(lam):
    """From p_sigma = 0, p_sigma' = sqrt(c_s (2 - c_s) mu_eff) C^(-1/2) y_w has
    covariance c_s (2 - c_s) I for any C; from a stationary N(0, I) draw it
    stays N(0, I)."""
    n = 9
    r, _, k = _random_selection_trials(n, lam, False, False)
    cs = k["c_sigma"]
    cov = np.cov(r["ps"].T) / (cs * (2.0 - cs))
    assert np.all(np.abs(cov - np.eye(n)) <= _cov_bound(np.eye(n), N_TRIALS))
    r2, _, _ = _random_selection_trials(n, lam, True, False, seed=321)
    cov2 = np.cov(r2["ps"].T)
    assert np.all(np.abs(cov2 - np.eye(n)) <= _cov_bound(np.eye(n), N_TRIALS))
    assert np.all(np.abs(r2["ps"].mean(0)) <= 5.0 / math.sqrt(N_TRIALS))


@pytest.mark.parametrize("lam", [16, 70])
def test_random_selection_covariance_is_unbiased(lam):
    """With p_c in its stationary law N(0, C) and p_sigma = 0 (so h_sigma = 1),
    E[C'] = C: the rank-one and rank-mu terms replace exactly what the decay
    (1 - c_1 - c_mu sum w) removes."""
    n = 9
    r, C, k = _random_selection_trials(n, lam, False, True)
    mean_C = r["C"].mean(0)
    d = np.sqrt(np.diag(C))
    per_trial_var = (k["c_mu"] ** 2 / k["mu_eff"] + k["c1"] ** 2) * (np.outer(d, d) ** 2 + C ** 2)
    assert np.all(np.abs(mean_C - C) <= 5.0 * np.sqrt(per_trial_var / N_TRIALS))
    # the bound is tight enough to see a dropped rank-one term (its mean is c_1 C)
    # or a decay off by c_1
    assert 5.0 * np.sqrt(per_trial_var.max() / N_TRIALS) < 0.5 * k["c1"] * np.abs(C).max()


def test_random_selection_log_step_size_has_zero_drift():
    """With p_sigma stationary, ||p_sigma'|| is chi-distributed with n degrees of
    freedom, so E[ln sigma' - ln sigma] = (c_s / d_s)(E chi_n / chi_n_approx - 1),
    which is below 1e-4 for n = 9 (E chi_n = sqrt 2 Gamma((n+1)/2) / Gamma(n/2))."""
    n, lam = 9, 16
    r, _, k = _random_selection_trials(n, lam, True, False, seed=77)
    e_chi = math.sqrt(2.0) * math.exp(math.lgamma((n + 1) / 2.0) - math.lgamma(n / 2.0))
    drift = k["c_sigma"] / k["d_sigma"] * (e_chi / k["chi_n"] - 1.0)
    assert abs(drift) < 1e-4
    d = r["dlogs"]
    assert abs(d.mean() - drift) <= 5.0 * d.std() / math.sqrt(N_TRIALS)
    # and the spread is that of a chi variable scaled by c_s / (d_s chi_n)
    chi_var = n - e_chi ** 2
    np.testing.assert_allclose(d.std(), k["c_sigma"] / k["d_sigma"] * math.sqrt(chi_var) / k["chi_n"], rtol=0.1)
