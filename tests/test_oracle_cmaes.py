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
