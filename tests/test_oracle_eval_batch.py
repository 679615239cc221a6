"""Pin of the oracle's batch evaluator (the CPU baseline's fitness step).

tko_eval_batch runs forward kinematics (Sec. III-A.3), projection and snap,
the integer rasteriser (renderer of Eq. (7), OR over the arms for the joint
bi-manual image of Sec. III-B) and the counts |S|, |S and M| of Eq. (6) for
many candidates, with OpenMP over candidates.  Its counts and masks must be
those of the single-candidate path (fk -> project_snap -> raster -> counts,
each pinned on its own by closed forms), whatever the thread count: a
candidate or arm offset slip, a missing OR across arms or a race between
threads shows up as a mismatch here.
"""
import numpy as np
import pytest

import oracle
import scenes


def _single(theta_row, chains, meshes, cam, target):
    mask = oracle.render(theta_row, chains, meshes, cam)
    a, i, _ = oracle.counts(mask, target, cam.width, cam.height)
    return mask, (a, i)


def _case(n_arms, B, seed):
    rng = np.random.default_rng(seed)
    cam = scenes.camera(96, 72, f=120.0)
    meshes = [scenes.instrument_mesh(12, 4, 1, 1), scenes.instrument_mesh(10, 3, 1, 1, jaw_scale=1.3)][:n_arms]
    chains = [scenes.chain(), scenes.chain(jaw_scale=1.3)][:n_arms]
    base = np.concatenate([scenes.true_pose(rng, cam) for _ in range(n_arms)])
    scale = np.tile(scenes.DEFAULT_SCALE, n_arms)
    theta = base[None, :] + 2.0 * scale[None, :] * rng.normal(size=(B, 9 * n_arms))
    theta[3] = np.nan                              # a candidate that is not a number: empty silhouette
    theta[5, 5] = -0.05                            # first arm behind the camera (all its vertices culled)
    target = oracle.render(base, chains, meshes, cam)
    flips = scenes.flip_indices(rng, cam.width, cam.height, fraction=0.05)
    target = scenes.apply_flips(target, cam.width, cam.height, flips)
    return theta, chains, meshes, cam, target


@pytest.mark.parametrize("n_arms", [1, 2])
@pytest.mark.parametrize("threads", [1, 0])
def test_eval_batch_equals_single_candidate_path(n_arms, threads):
    B = 24
    theta, chains, meshes, cam, target = _case(n_arms, B, seed=40 + n_arms)
    cnt, masks = oracle.eval_batch(theta, chains, meshes, cam, target, n_threads=threads, want_masks=True)
    assert cnt.shape == (B, 2) and masks.shape[0] == B
    nonempty = 0
    for k in range(B):
        mk, (a, i) = _single(theta[k], chains, meshes, cam, target)
        assert np.array_equal(masks[k], mk), f"candidate {k}: mask differs"
        assert (int(cnt[k, 0]), int(cnt[k, 1])) == (a, i), f"candidate {k}: counts {cnt[k]} vs {(a, i)}"
        nonempty += a > 0
    assert tuple(cnt[3]) == (0, 0)                 # NaN candidate
    assert nonempty >= B // 2                      # the comparison is not vacuous


def test_eval_batch_two_arms_is_the_union():
    """Two arms: the batch mask is the OR of the single-arm renders, and its
    count exceeds each arm's alone somewhere (the arms do not coincide)."""
    B = 6
    theta, chains, meshes, cam, target = _case(2, B, seed=7)
    _, masks = oracle.eval_batch(theta, chains, meshes, cam, target, n_threads=2, want_masks=True)
    grew = False
    for k in range(B):
        m0 = oracle.render(theta[k, :9], chains[:1], meshes[:1], cam)
        m1 = oracle.render(theta[k, 9:], chains[1:], meshes[1:], cam)
        assert np.array_equal(masks[k], m0 | m1)
        pop = lambda w: int(sum(bin(int(x)).count("1") for x in w.ravel()))
        grew |= pop(masks[k]) > max(pop(m0), pop(m1))
    assert grew


def test_eval_batch_thread_counts_agree():
    B = 40
    theta, chains, meshes, cam, target = _case(1, B, seed=3)
    ref = oracle.eval_batch(theta, chains, meshes, cam, target, n_threads=1)
    for t in (2, 3, oracle.max_threads()):
        assert np.array_equal(oracle.eval_batch(theta, chains, meshes, cam, target, n_threads=t), ref)
