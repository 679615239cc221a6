"""Pins of the Kalman-filter oracle (Sec. III-A.4): the steady-state predicted
covariance equals the discrete algebraic Riccati solution computed by scipy,
R -> 0 passes the measurement through, R -> inf keeps the constant-velocity
prediction, noiseless constant-velocity motion is tracked exactly, the
covariance stays symmetric, and the clamp holds the limits."""
import numpy as np
import scipy.linalg

from oracle.kalman import KalmanCV


def test_steady_state_matches_riccati():
    n, dt = 3, 1.0
    q_pos, q_vel, r = np.array([1e-4, 2e-4, 5e-5]), np.array([1e-5, 3e-5, 2e-5]), np.array([1e-3, 5e-4, 2e-3])
    kf = KalmanCV.diagonal(np.zeros(n), 1.0, 1.0, q_pos, q_vel, r, dt)
    for _ in range(2000):
        kf.step(np.zeros(n))
    # predicted covariance P- of the steady state solves the filtering DARE:
    # P = F P F^T - F P H^T (H P H^T + R)^-1 H P F^T + Q
    X = scipy.linalg.solve_discrete_are(kf.F.T, kf.H.T, kf.Q, kf.R)
    P_pred = kf.F @ kf.P @ kf.F.T + kf.Q
    np.testing.assert_allclose(P_pred, X, rtol=1e-8, atol=1e-14)


def test_tiny_measurement_noise_passes_measurement():
    kf = KalmanCV.diagonal(np.zeros(2), 1.0, 1.0, 1e-2, 1e-2, 1e-18)
    rng = np.random.default_rng(0)
    for _ in range(5):
        z = rng.normal(size=2)
        np.testing.assert_allclose(kf.step(z), z, atol=1e-12)


def test_huge_measurement_noise_keeps_prediction():
    kf = KalmanCV.diagonal(np.array([1.0, -2.0]), 1e-6, 1e-6, 0.0, 0.0, 1e18, dt=0.5)
    kf.s[2:] = [0.2, 0.4]                     # velocities
    th = kf.step(np.array([100.0, 100.0]))
    np.testing.assert_allclose(th, [1.0 + 0.5 * 0.2, -2.0 + 0.5 * 0.4], atol=1e-9)


def test_constant_velocity_is_tracked_exactly():
    n = 4
    x0, v = np.array([0.1, -0.3, 2.0, 0.5]), np.array([0.01, 0.02, -0.03, 0.0])
    kf = KalmanCV.diagonal(x0 + 0.05, 1.0, 1.0, 1e-12, 1e-12, 1e-6)
    for t in range(1, 300):
        est = kf.step(x0 + v * t)
    np.testing.assert_allclose(est, x0 + v * 299, atol=1e-6)
    np.testing.assert_allclose(kf.s[n:], v, atol=1e-7)
    np.testing.assert_allclose(kf.P, kf.P.T, atol=0)


def test_clamp_holds_limits():
    lo, hi = np.array([-1.0, -np.inf]), np.array([1.0, np.inf])
    kf = KalmanCV.diagonal(np.zeros(2), 1.0, 1.0, 1e-2, 1e-2, 1e-6, lo=lo, hi=hi)
    th = kf.step(np.array([5.0, 5.0]))
    assert th[0] == 1.0 and abs(th[1] - 5.0) < 1e-3


def test_missing_measurement_is_pure_prediction():
    kf = KalmanCV.diagonal(np.array([0.0, 1.0]), 1.0, 1.0, 1e-3, 1e-3, 1e-2, dt=0.5)
    kf.step(np.array([0.2, 1.1]))
    s_prev, P_prev = kf.s.copy(), kf.P.copy()
    th = kf.step(np.array([np.nan, 1.3]))
    # the unobserved coordinate follows the motion model alone
    s_pred = kf.F @ s_prev
    P_pred = kf.F @ P_prev @ kf.F.T + kf.Q
    assert th[0] == s_pred[0] and kf.s[2] == s_pred[2]
    np.testing.assert_allclose(kf.P[0, 0], P_pred[0, 0], rtol=1e-15)
    assert abs(th[1] - 1.3) < abs(s_pred[1] - 1.3)


def test_decoupled_scalar_filters_equal_joint_filter():
    """With block-diagonal noise the 2n filter separates: running each
    coordinate as its own 2-state filter gives the same trajectory."""
    rng = np.random.default_rng(3)
    n, dt = 5, 0.04
    qp, qc, qv, r = rng.uniform(1e-5, 1e-3, n), rng.uniform(-1e-6, 1e-6, n), rng.uniform(1e-4, 1e-2, n), \
        rng.uniform(1e-4, 1e-2, n)
    x0 = rng.normal(size=n)
    joint = KalmanCV.diagonal(x0, 0.1, 1.0, qp, qv, r, dt, q_cross=qc)
    single = [KalmanCV.diagonal(x0[i:i + 1], 0.1, 1.0, qp[i], qv[i], r[i], dt, q_cross=qc[i]) for i in range(n)]
    for t in range(50):
        z = x0 + 0.3 * np.sin(0.1 * t + np.arange(n)) + 0.01 * rng.normal(size=n)
        a = joint.step(z)
        b = np.array([single[i].step(z[i:i + 1])[0] for i in range(n)])
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def test_scalar_random_walk_gain_closed_form():
    """dt-free special case: velocity noise 0 and zero initial velocity
    variance reduce the filter to a scalar random walk, whose steady-state
    prior variance solves p = p r / (p + r) + q, i.e. p = (q + sqrt(q^2 + 4 q r)) / 2."""
    q, r = 2e-3, 5e-2
    kf = KalmanCV.diagonal(np.zeros(1), 1.0, 0.0, q, 0.0, r, dt=1.0)
    for _ in range(500):
        kf.step(np.zeros(1))
    p_prior = kf.P[0, 0] + q
    np.testing.assert_allclose(p_prior, (q + np.sqrt(q * q + 4 * q * r)) / 2, rtol=1e-12)
