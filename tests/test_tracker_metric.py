"""Host logic of the pose-error metric (Sec. IV, evaluation metrics): of the
two equivalent solutions of the instrument's symmetry, the truth and
(beta + pi, -q1, -q2, q3), the one with the smaller absolute roll error is
scored.  (That the two render the same silhouette is pinned on the oracle by
the roll-by-pi symmetry test.)"""
import numpy as np

from paper_2603_11404_amd.tracker import symmetric_reference


def _truth(rng, F, arms):
    t = np.zeros((F, 9 * arms))
    for a in range(arms):
        o = 9 * a
        t[:, o:o + 3] = rng.uniform(-np.pi, np.pi, (F, 3))
        t[:, o + 3:o + 6] = rng.normal(size=(F, 3)) * 0.01
        t[:, o + 6:o + 8] = rng.uniform(-1.2, 1.2, (F, 2))
        t[:, o + 8] = rng.uniform(0.1, 1.4, F)
    return t


def _equivalent(t, arms):
    e = t.copy()
    for a in range(arms):
        o = 9 * a
        e[:, o + 1] += np.pi
        e[:, o + 6:o + 8] *= -1.0
    return e


def test_estimate_near_truth_keeps_truth():
    rng = np.random.default_rng(0)
    t = _truth(rng, 50, 1)
    est = t + rng.normal(size=t.shape) * 0.05
    ref, flipped = symmetric_reference(est, t, 1)
    assert not flipped.any()
    assert np.array_equal(ref, t)


def test_estimate_at_the_equivalent_scores_the_equivalent():
    rng = np.random.default_rng(1)
    t = _truth(rng, 50, 1)
    eq = _equivalent(t, 1)
    est = eq + rng.normal(size=t.shape) * 0.05
    ref, flipped = symmetric_reference(est, t, 1)
    assert flipped.all()
    np.testing.assert_array_equal(ref, eq)
    # the scored joint and roll errors are the small ones
    assert np.abs(est[:, 6:8] - ref[:, 6:8]).max() < 0.3
    assert np.abs(np.angle(np.exp(1j * (est[:, 1] - ref[:, 1])))).max() < 0.3


def test_roll_compared_modulo_two_pi():
    t = np.zeros((3, 9))
    t[:, 1] = [np.pi - 0.01, -np.pi + 0.01, 0.4]
    est = t.copy()
    est[:, 1] = [-np.pi + 0.02, np.pi - 0.02, 0.4 + np.pi - 0.05 - 2 * np.pi]   # wrap-around, equivalent
    _, flipped = symmetric_reference(est, t, 1)
    assert list(flipped[:, 0]) == [False, False, True]


def test_arms_resolved_independently():
    rng = np.random.default_rng(2)
    t = _truth(rng, 20, 2)
    est = t.copy()
    est[:, 9:] = _equivalent(t, 2)[:, 9:]        # second arm at its equivalent only
    ref, flipped = symmetric_reference(est, t, 2)
    assert not flipped[:, 0].any() and flipped[:, 1].all()
    np.testing.assert_array_equal(ref[:, :9], t[:, :9])
    np.testing.assert_array_equal(ref[:, 9:], est[:, 9:])
