"""Pins of the oracle's counts and losses (Eq. render_loss, mask error 1 - IoU of
Sec. IV, keypoint term Eq. kpts_loss)."""
import math

import numpy as np
import pytest

import oracle
import scenes

CH = scenes.chain()


def _popcount(words):
    w = np.asarray(words, dtype=np.uint64)
    return int(sum(bin(int(x)).count("1") for x in w.ravel()))


def test_counts_match_bitcount_brute_force():
    rng = np.random.default_rng(11)
    for W, H in [(320, 240), (13, 9), (64, 8)]:
        S = scenes.image_to_words(rng.random((H, W)) < 0.3)
        M = scenes.image_to_words(rng.random((H, W)) < 0.4)
        a, i, m = oracle.counts(S, M, W, H)
        assert a == _popcount(S) and m == _popcount(M) and i == _popcount(S & M)


def test_self_iou_and_empty():
    wl = scenes.workload("small")
    mesh, cam = wl["mesh"], wl["cam"]
    th = scenes.true_pose(scenes.rng_for(0, 0), cam)
    S = oracle.render(th, [CH], [mesh], cam)
    a, i, m = oracle.counts(S, S, cam.width, cam.height)
    assert a == i == m > 0
    assert oracle.mask_loss(a, i, m, kind=0) == 0.0                   # IoU(S, S) = 1
    empty = np.zeros_like(S)
    a, i, m = oracle.counts(S, empty, cam.width, cam.height)
    assert i == 0 and m == 0 and oracle.mask_loss(a, i, m, kind=0) == 1.0   # IoU(S, 0) = 0
    assert oracle.mask_loss(0, 0, 0, kind=0) == 0.0                   # empty union: IoU := 1


def test_flips_give_exact_xor_count():
    """At the true pose the rendered mask differs from the flipped target in
    exactly the flipped pixels (Eq. render_loss squared error = xor count)."""
    wl = scenes.workload("small")
    mesh, cam = wl["mesh"], wl["cam"]
    th = scenes.true_pose(scenes.rng_for(0, 0), cam)
    S = oracle.render(th, [CH], [mesh], cam)
    idx = scenes.flip_indices(scenes.rng_for(0, scenes.SUB_FLIPS), cam.width, cam.height)
    assert len(idx) == 768
    T = scenes.apply_flips(S, cam.width, cam.height, idx)
    a, i, m = oracle.counts(S, T, cam.width, cam.height)
    img = scenes.words_to_image(S, cam.width, cam.height).ravel()
    f_in = int(img[idx].sum())
    assert a + m - 2 * i == 768
    assert i == a - f_in
    assert oracle.mask_loss(a, i, m, kind=1, lambda_app=0.0) == 768.0
    assert oracle.mask_loss(a, i, m, kind=1, lambda_app=2.0) == 768.0 + 2.0 * abs(a - m)


def test_iou_on_hand_example():
    W, H = 8, 8
    S = np.zeros((H, W), bool)
    S[0:2, 0:4] = True         # 8 px
    M = np.zeros((H, W), bool)
    M[1:3, 2:6] = True         # 8 px, overlap 2 px
    a, i, m = oracle.counts(scenes.image_to_words(S), scenes.image_to_words(M), W, H)
    assert (a, i, m) == (8, 2, 8)
    assert oracle.mask_loss(a, i, m, 0) == pytest.approx(1 - 2 / 14, abs=1e-15)
    assert oracle.mask_loss(a, i, m, 1, 0.5) == 12.0


def test_keypoint_loss_properties():
    rng = np.random.default_rng(12)
    ref = rng.uniform(0, 600, size=(4, 2))
    assert oracle.kp_loss(ref, ref) == 0.0
    # swapping the two jaw tips of the prediction does not change the loss
    kp = ref + rng.normal(size=(4, 2)) * 3
    sw = kp[[0, 1, 3, 2]]
    assert oracle.kp_loss(kp, ref) == pytest.approx(oracle.kp_loss(sw, ref), abs=1e-12)
    # one fixed keypoint displaced by (3, 4) px, tau = 0 -> 5 px
    kp = ref.copy()
    kp[0] += [3.0, 4.0]
    assert oracle.kp_loss(kp, ref) == pytest.approx(5.0, abs=1e-12)
    # the threshold tau removes errors smaller than it
    assert oracle.kp_loss(kp, ref, tau=6.0) == 0.0
    # both tips shifted by (1, 0): two tip terms of 1 plus the midpoint term of 1
    kp = ref.copy()
    kp[2:] += [1.0, 0.0]
    assert oracle.kp_loss(kp, ref) == pytest.approx(3.0, abs=1e-12)
    kp = ref.copy()
    kp[1] = [math.nan, math.nan]
    assert math.isnan(oracle.kp_loss(kp, ref))


def test_two_tip_keypoint_loss_of_the_paper():
    """Eq. (8) on the two tool tips: worked values, symmetry in the order of
    the detected tips, the tau threshold, the midpoint term, and the skip rule
    (no term unless two distinct reference tips exist)."""
    import math
    ref = np.array([[0.0, 0.0], [0.0, 0.0], [10.0, 20.0], [30.0, 20.0]])
    kp = ref.copy()
    assert oracle.kp_loss_tips(kp, ref) == 0.0
    kp_sw = kp.copy()
    kp_sw[[2, 3]] = kp[[3, 2]]                         # detections in the other order
    assert oracle.kp_loss_tips(kp_sw, ref) == 0.0
    # both tips moved by (3, 4): |v| = 5 each and for the midpoint
    kp_v = kp.copy()
    kp_v[2:] += [3.0, 4.0]
    assert oracle.kp_loss_tips(kp_v, ref) == pytest.approx(15.0, abs=1e-12)
    assert oracle.kp_loss_tips(kp_v, ref, tau=1.0) == pytest.approx(12.0, abs=1e-12)
    assert oracle.kp_loss_tips(kp_v, ref, tau=6.0) == 0.0
    # one tip moved by 6 along x: the tips term is 6, the midpoint moves by 3
    kp_1 = kp.copy()
    kp_1[3, 0] += 6.0
    assert oracle.kp_loss_tips(kp_1, ref) == pytest.approx(9.0, abs=1e-12)
    # the better assignment is taken: tips crossed over and shifted
    kp_x = kp.copy()
    kp_x[2], kp_x[3] = ref[3] + [0.0, 1.0], ref[2] + [0.0, 1.0]
    assert oracle.kp_loss_tips(kp_x, ref) == pytest.approx(2.0 + 1.0, abs=1e-12)
    # shaft and wrist keypoints play no part
    kp_o = kp_v.copy()
    kp_o[0:2] += 100.0
    assert oracle.kp_loss_tips(kp_o, ref) == oracle.kp_loss_tips(kp_v, ref)
    # skip rule: a missing or a coincident reference tip
    ref_nan = ref.copy()
    ref_nan[3, 1] = math.nan
    assert oracle.kp_loss_tips(kp_v, ref_nan) == 0.0
    ref_same = ref.copy()
    ref_same[3] = ref[2]
    assert oracle.kp_loss_tips(kp_v, ref_same) == 0.0
    # a candidate tip behind the camera (NaN) makes the loss NaN (ranked last)
    kp_nan = kp.copy()
    kp_nan[2, 0] = math.nan
    assert math.isnan(oracle.kp_loss_tips(kp_nan, ref))
