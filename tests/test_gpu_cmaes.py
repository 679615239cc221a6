"""GPU parity of the FP64 CMA-ES kernels against the numpy oracle.

Given the same state (the oracle's m, sigma, C, L, p_sigma, p_c, g written into
the device blob, with its B as the Jacobi warm start) and the same losses,
sampling and update agree to 1e-12, the new Cholesky factor L included (it is
unique); eigen-decompositions are compared through invariants (reconstruction
of the covariance they were taken of, orthonormality, eigenvalues) since
eigenvector order and signs are not unique.
"""
import numpy as np
import pytest
import torch

from oracle import cmaes

pytestmark = pytest.mark.gpu
DEV = "cuda"


def tk():
    from paper_2603_11404_amd import tk as _tk
    return _tk


def _pair(n, lam, seed=5, n_blocks=1, sigma0=0.8):
    T = tk()
    rng = np.random.default_rng(seed)
    m0 = rng.normal(size=n)
    off = rng.normal(size=n)
    sc = rng.uniform(0.01, 0.2, n)
    es = cmaes.CMAES(n, lam, m0, sigma0, off, sc, seed, n_blocks=n_blocks)
    st = T.cmaes_alloc(n, lam, DEV)
    T.cmaes_init(st, n, lam, m0, sigma0, off, sc, seed, n_blocks=n_blocks)
    return es, st


def _push(es, st, n, lam):
    tk().cmaes_write(st, n, lam, mean=es.m, sigma=[es.sigma], C=es.C, L=es.L, B=es.B, D=es.D, p_sigma=es.p_sigma,
                     p_c=es.p_c, gen=es.g)


@pytest.mark.parametrize("n,lam", [(9, 16), (9, 256), (18, 512), (3, 70), (18, 1024)])
def test_init_constants(n, lam):
    es, st = _pair(n, lam)
    torch.cuda.synchronize()
    v = tk().cmaes_view(st, n, lam)
    for key in ("mu_eff", "c_sigma", "d_sigma", "c_c", "c1", "c_mu", "c_m", "chi_n"):
        assert v[key] == pytest.approx(es.k[key], rel=1e-13), key
    np.testing.assert_allclose(v["weights"][:lam // 2], es.k["weights"], rtol=1e-13)
    assert np.all(v["weights"][lam // 2:] == 0)
    np.testing.assert_array_equal(v["C"], np.eye(n))
    np.testing.assert_array_equal(v["L"], np.eye(n))
    assert v["gen"] == 0 and v["flags"] == 0


@pytest.mark.parametrize("n,lam,nb", [(9, 16, 1), (9, 256, 1), (18, 512, 2)])
def test_sample_matches_oracle_given_state(n, lam, nb):
    T = tk()
    es, st = _pair(n, lam, n_blocks=nb)
    rng = np.random.default_rng(9)
    for g in range(3):
        # a non-trivial state from the oracle itself
        es.update(rng.normal(size=lam)) if es.Y is not None else None
        _push(es, st, n, lam)
        theta = es.sample()
        X = torch.empty(lam, n, dtype=torch.float32, device=DEV)
        T.cmaes_sample(st, n, lam, X)
        torch.cuda.synchronize()
        v = T.cmaes_view(st, n, lam)
        np.testing.assert_allclose(v["Z"], es.Z, rtol=0, atol=1e-13)
        np.testing.assert_allclose(v["Y"], es.Y, rtol=0, atol=1e-12 * max(1.0, np.abs(es.Y).max()))
        Xg = X.cpu().numpy()
        np.testing.assert_allclose(Xg, theta.astype(np.float32), rtol=2e-7, atol=1e-7)


@pytest.mark.parametrize("n,lam,nb", [(9, 16, 1), (9, 256, 1), (18, 512, 2), (18, 64, 1), (9, 1024, 1), (18, 1024, 2)])
def test_update_matches_oracle_given_state(n, lam, nb):
    T = tk()
    es, st = _pair(n, lam, n_blocks=nb)
    rng = np.random.default_rng(11)
    A = rng.normal(size=(n, n))
    H = A @ A.T + np.eye(n)
    for g in range(4):
        _push(es, st, n, lam)
        X = torch.empty(lam, n, dtype=torch.float32, device=DEV)
        T.cmaes_sample(st, n, lam, X)
        theta = es.sample()
        x = (theta - es.offset) / es.scale
        loss = np.einsum("ki,ij,kj->k", x, H, x)
        loss[3] = np.nan
        loss[5] = loss[6]                     # a tie
        # the GPU keeps its own Y (equal to the oracle's within 1e-12); feed the same losses
        lt = torch.as_tensor(loss, device=DEV)
        C_old = es.C.copy()
        es.update(loss)
        T.cmaes_update(st, n, lam, lt)
        torch.cuda.synchronize()
        v = T.cmaes_view(st, n, lam)
        np.testing.assert_array_equal(v["order"], cmaes.CMAES.ranking(loss))
        tol = 1e-11
        np.testing.assert_allclose(v["mean"], es.m, rtol=0, atol=tol)
        assert v["sigma"] == pytest.approx(es.sigma, rel=1e-12)
        np.testing.assert_allclose(v["p_sigma"], es.p_sigma, rtol=0, atol=tol)
        np.testing.assert_allclose(v["p_c"], es.p_c, rtol=0, atol=tol)
        np.testing.assert_allclose(v["C"], es.C, rtol=0, atol=tol * np.abs(C_old).max())
        assert v["gen"] == es.g and v["h_sigma"] == es.h_sigma
        # the sampling factor of the new covariance: the oracle's (unique) Cholesky factor
        Lg = v["L"]
        assert np.all(np.triu(Lg, 1) == 0.0) and np.all(np.diag(Lg) > 0)
        np.testing.assert_allclose(Lg, es.L, rtol=0, atol=tol * np.sqrt(np.abs(C_old).max()))
        np.testing.assert_allclose(Lg @ Lg.T, v["C"], rtol=0, atol=1e-13 * np.abs(v["C"]).max())
        # eigen-decomposition of the covariance the candidates were drawn with
        B, D = v["B"], v["D"]
        np.testing.assert_allclose(B.T @ B, np.eye(n), atol=1e-13)
        np.testing.assert_allclose(B @ np.diag(D ** 2) @ B.T, C_old, atol=1e-12 * np.abs(C_old).max())
        np.testing.assert_allclose(np.sort(D), np.sort(es.D), rtol=1e-10)
        assert v["flags"] == 0
        if nb > 1:
            assert np.all(v["C"][:9, 9:] == 0) and np.all(B[:9, 9:] == 0) and np.all(B[9:, :9] == 0)
            assert np.all(Lg[:9, 9:] == 0) and np.all(Lg[9:, :9] == 0)


def _one_update(es, st, n, lam, loss_fn):
    T = tk()
    _push(es, st, n, lam)
    X = torch.empty(lam, n, dtype=torch.float32, device=DEV)
    T.cmaes_sample(st, n, lam, X)
    theta = es.sample()
    loss = loss_fn((theta - es.offset) / es.scale)
    C_old = es.C.copy()
    es.update(loss)
    T.cmaes_update(st, n, lam, torch.as_tensor(loss, device=DEV))
    torch.cuda.synchronize()
    return T.cmaes_view(st, n, lam), C_old


@pytest.mark.parametrize("n,lam,nb", [(9, 256, 1), (18, 512, 2)])
def test_update_with_h_sigma_zero_matches_oracle(n, lam, nb):
    """A long conjugate path makes h_sigma = 0: the covariance and its factor
    are then formed with the h_sigma correction (not the h_sigma = 1 form the
    update prepares beside the eigendecomposition)."""
    es, st = _pair(n, lam, n_blocks=nb)
    es.p_sigma = np.full(n, 50.0)
    es.p_c = np.linspace(-1.0, 1.0, n)
    v, C_old = _one_update(es, st, n, lam, lambda x: np.sum(x * x, 1))
    assert es.h_sigma == 0.0 and v["h_sigma"] == 0.0
    tol = 1e-11
    np.testing.assert_allclose(v["p_c"], es.p_c, rtol=0, atol=tol)
    np.testing.assert_allclose(v["C"], es.C, rtol=0, atol=tol * np.abs(C_old).max())
    np.testing.assert_allclose(v["L"], es.L, rtol=0, atol=tol)
    assert v["sigma"] == pytest.approx(es.sigma, rel=1e-12)


def test_update_floors_a_singular_covariance_like_the_oracle():
    """C = diag(1, ..., 1, 0): its zero Cholesky pivot is floored, so the draws
    reach that direction only at the floor's scale and the new covariance's
    last pivot stays below its floor.  The zero eigenvalue and the pivots are
    floored at 1e-20 of the largest, as in the oracle, and the flag says so."""
    n, lam = 9, 16
    es, st = _pair(n, lam)
    C = np.eye(n)
    C[n - 1, n - 1] = 0.0
    es.set_covariance(C)
    assert es.chol_floored
    v, C_old = _one_update(es, st, n, lam, lambda x: np.sum(x * x, 1))
    assert es.eig_floored and es.chol_floored
    assert v["flags"] & 1
    np.testing.assert_allclose(v["mean"], es.m, rtol=0, atol=1e-11)
    np.testing.assert_allclose(v["C"], es.C, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v["L"], es.L, rtol=0, atol=1e-11)
    floor = 1e-20 * np.max(np.diag(es.C))
    assert v["C"][n - 1, n - 1] < floor
    assert v["L"][n - 1, n - 1] == pytest.approx(np.sqrt(floor), rel=1e-12)


def _gpu_run(fun, n=9, lam=16, gens=200, seed=1, m0=3.0):
    T = tk()
    st = T.cmaes_alloc(n, lam, DEV)
    T.cmaes_init(st, n, lam, np.full(n, m0), 1.0, np.zeros(n), np.ones(n), seed)
    X = torch.empty(lam, n, dtype=torch.float32, device=DEV)
    hist = []
    for g in range(gens):
        T.cmaes_sample(st, n, lam, X)
        T.cmaes_update(st, n, lam, fun(X.double()))
        v = T.cmaes_view(st, n, lam)
        hist.append(v)
    return hist


def test_sphere_converges_on_gpu():
    """Same bound as the oracle pin: f(m) <= 1e-10 within 180 generations (n = 9,
    lambda = 16, m0 = 3, sigma0 = 1).  Candidates pass through FP32, so the
    threshold is on the FP64 mean the update keeps."""
    for seed in range(4):
        T = tk()
        n, lam = 9, 16
        st = T.cmaes_alloc(n, lam, DEV)
        T.cmaes_init(st, n, lam, np.full(n, 3.0), 1.0, np.zeros(n), np.ones(n), seed)
        X = torch.empty(lam, n, dtype=torch.float32, device=DEV)
        Y = None
        done = False
        for g in range(180):
            T.cmaes_sample(st, n, lam, X)
            L = T.cmaes_layout(n, lam)
            # loss from the FP64 draws kept in the state: f(x) = |m + sigma y|^2
            raw = st[L["Y"]:L["Y"] + 8 * lam * n].view(torch.float64).view(lam, n)
            mean = st[L["mean"]:L["mean"] + 8 * n].view(torch.float64)
            sigma = st[L["sigma"]:L["sigma"] + 8].view(torch.float64)
            x = mean[None, :] + sigma * raw
            T.cmaes_update(st, n, lam, (x * x).sum(1).contiguous())
            if g % 10 == 9:
                m = T.cmaes_view(st, n, lam)["mean"]
                if float(np.sum(m ** 2)) <= 1e-10:
                    done = True
                    break
        assert done, f"seed {seed} did not converge"
        del Y


def test_ranking_invariance_bit_identical_on_gpu():
    h1 = _gpu_run(lambda X: (X * X).sum(1).contiguous(), gens=25)
    h2 = _gpu_run(lambda X: (torch.exp(torch.sqrt((X * X).sum(1))) * 5 + 1).contiguous(), gens=25)
    for a, b in zip(h1, h2):
        assert np.array_equal(a["mean"], b["mean"]) and a["sigma"] == b["sigma"]
        assert np.array_equal(a["C"], b["C"]) and np.array_equal(a["B"], b["B"])


def test_deterministic_double_run():
    h1 = _gpu_run(lambda X: (X * X).sum(1).contiguous(), gens=10, seed=3)
    h2 = _gpu_run(lambda X: (X * X).sum(1).contiguous(), gens=10, seed=3)
    for a, b in zip(h1, h2):
        for k in ("mean", "C", "L", "B", "D", "Z", "Y", "p_sigma", "p_c"):
            assert np.array_equal(a[k], b[k]), k


def test_cmaes_argument_errors():
    T = tk()
    st = T.cmaes_alloc(9, 16, DEV)
    with pytest.raises(T.TkError):
        T.cmaes_init(st, 9, 16, np.zeros(9), -1.0, np.zeros(9), np.ones(9), 0)
    with pytest.raises(T.TkError):
        T.cmaes_init(st, 9, 16, np.zeros(9), 1.0, np.zeros(9), np.ones(9), 0, n_blocks=2)
    with pytest.raises(T.TkError):
        T.cmaes_sample(st[1:], 9, 16, torch.empty(16, 9, device=DEV))   # misaligned state
