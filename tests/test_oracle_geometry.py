"""Pins of the oracle's geometry: cosine joint map, look-at pose, chain, projection.

Each check uses a fact fixed by the paper or by geometry, not a retyped formula:
limits of the cosine map (Sec. III-A.3), the look-at decoupling of beta from the
shaft axis (Sec. III-A.3), right-hand-rule images of basis vectors, 2*pi
periodicity, the instrument's 180-degree symmetry (Sec. III-A.3), and the
pinhole principal point.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

CH = scenes.chain()


# ------------------------------------------------------------ cosine joint map

@pytest.mark.parametrize("lb,ub", [(-math.pi / 2, math.pi / 2), (0.0, math.pi / 2), (-0.3, 1.7)])
def test_decode_limits_and_range(lb, ub):
    assert oracle.decode(lb, lb, ub) == pytest.approx(lb, abs=1e-15)
    assert oracle.decode(ub, lb, ub) == pytest.approx(ub, abs=1e-14)
    # every unconstrained value maps inside the box (the point of the reparameterisation)
    for qh in np.linspace(-50, 50, 2001):
        q = oracle.decode(qh, lb, ub)
        assert lb - 1e-15 <= q <= ub + 1e-15
    # midpoint maps to midpoint, and the map is periodic with period 2(ub-lb)
    mid = 0.5 * (lb + ub)
    assert oracle.decode(mid, lb, ub) == pytest.approx(mid, abs=1e-14)
    assert oracle.decode(0.37 + 2 * (ub - lb), lb, ub) == pytest.approx(oracle.decode(0.37, lb, ub), abs=1e-13)


@pytest.mark.parametrize("lb,ub", [(-math.pi / 2, math.pi / 2), (0.0, math.pi / 2)])
def test_encode_inverts_decode(lb, ub):
    for q in np.linspace(lb, ub, 101):
        assert oracle.decode(oracle.encode(q, lb, ub), lb, ub) == pytest.approx(q, abs=1e-12)
        qh = oracle.encode(q, lb, ub)
        assert lb - 1e-12 <= qh <= ub + 1e-12       # encode lands in [lb, ub]


def test_decode_monotone_on_box():
    lb, ub = -math.pi / 2, math.pi / 2
    qs = [oracle.decode(x, lb, ub) for x in np.linspace(lb, ub, 500)]
    assert all(b > a for a, b in zip(qs, qs[1:]))


# ------------------------------------------------------------ look-at pose

def _R(a, b, g):
    return oracle.pose(a, b, g, 0, 0, 0)[:, :3]


def test_pose_identity_and_translation():
    T = oracle.pose(0, 0, 0, 0.1, -0.2, 0.3)
    np.testing.assert_array_equal(T[:, :3], np.eye(3))
    np.testing.assert_array_equal(T[:, 3], [0.1, -0.2, 0.3])


def test_single_axis_right_hand_rule():
    e = np.eye(3)
    # +90 deg about x sends +y to +z; about y sends +z to +x; about z sends +x to +y
    np.testing.assert_allclose(_R(math.pi / 2, 0, 0) @ e[1], e[2], atol=1e-15)
    np.testing.assert_allclose(_R(0, 0, math.pi / 2) @ e[2], e[0], atol=1e-15)
    np.testing.assert_allclose(_R(0, math.pi / 2, 0) @ e[0], e[1], atol=1e-15)
    # the rotation axis is fixed
    np.testing.assert_allclose(_R(0.7, 0, 0) @ e[0], e[0], atol=1e-15)
    np.testing.assert_allclose(_R(0, 0.7, 0) @ e[2], e[2], atol=1e-15)
    np.testing.assert_allclose(_R(0, 0, 0.7) @ e[1], e[1], atol=1e-15)


def test_rotation_orthonormal():
    rng = np.random.default_rng(1)
    for _ in range(200):
        R = _R(*rng.uniform(-7, 7, 3))
        np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-15)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-15)


def test_beta_is_roll_about_shaft_axis():
    """Look-at decoupling: beta only spins the instrument about its own z axis,
    so the image of e_z does not depend on beta, and beta composes additively."""
    rng = np.random.default_rng(2)
    for _ in range(100):
        a, g = rng.uniform(-3, 3, 2)
        b1, b2 = rng.uniform(-3, 3, 2)
        np.testing.assert_allclose(_R(a, b1, g) @ [0, 0, 1], _R(a, b2, g) @ [0, 0, 1], atol=1e-15)
        # R(a,b1+b2,g) = R(a,b1,g) * (rotation by b2 about the body z axis)
        Rz = _R(0, b2, 0)
        np.testing.assert_allclose(_R(a, b1 + b2, g), _R(a, b1, g) @ Rz, atol=1e-14)


def test_gamma_applies_last_about_camera_y():
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b, g = rng.uniform(-3, 3, 3)
        np.testing.assert_allclose(_R(a, b, g), _R(0, 0, g) @ _R(a, b, 0), atol=1e-14)
        np.testing.assert_allclose(_R(a, b, 0), _R(a, 0, 0) @ _R(0, b, 0), atol=1e-14)


# ------------------------------------------------------------ chain and FK

def test_fk_zero_state_is_identity_chain():
    th = np.zeros(9)
    th[6:9] = [0.0, 0.0, 0.0]
    # qhat = 0 decodes to q = 0 only for symmetric limits; jaw limits [0, pi/2] give q3 = 0 at qhat = 0
    M = oracle.fk(th, CH)
    np.testing.assert_allclose(M[0], np.eye(3, 4), atol=1e-15)
    np.testing.assert_allclose(M[1], np.eye(3, 4), atol=1e-15)
    jaw = np.eye(3, 4)
    jaw[2, 3] = CH.d_pitch_yaw
    np.testing.assert_allclose(M[2], jaw, atol=1e-15)
    np.testing.assert_allclose(M[3], jaw, atol=1e-15)


def test_jaw_opening_is_mirror_symmetric():
    q = [0.0, 0.0, 0.6]
    T = oracle.chain_links(q, CH)
    tip = np.array([0, 0, 0.014, 1.0])
    p_pos, p_neg = T[2] @ tip, T[3] @ tip
    assert p_pos[0] > 0 and p_neg[0] < 0                 # q3 opens jaw+ to +x, jaw- to -x
    np.testing.assert_allclose(p_pos * [-1, 1, 1], p_neg, atol=1e-15)
    # opening angle between the two jaws equals q3
    d1, d2 = T[2][:, 2], T[3][:, 2]
    assert math.acos(np.clip(d1 @ d2, -1, 1)) == pytest.approx(0.6, abs=1e-12)


def test_wrist_pitch_rotates_about_x():
    T = oracle.chain_links([0.4, 0.0, 0.0], CH)
    np.testing.assert_allclose(T[1][:, 0], [1, 0, 0], atol=1e-15)
    # yaw axis origin moves on the circle of radius d in the y-z plane
    o = T[2][:, 3]
    assert o[0] == pytest.approx(0, abs=1e-15)
    assert math.hypot(o[1], o[2]) == pytest.approx(CH.d_pitch_yaw, abs=1e-15)
    assert o[1] < 0                                   # Rx(+0.4) tilts +z towards -y


def test_two_pi_invariance_transforms_and_mask():
    wl = scenes.workload("small")
    mesh, cam = wl["mesh"], wl["cam"]
    th = scenes.true_pose(scenes.rng_for(0, 0), cam)
    M0 = oracle.fk(th, CH)
    m0 = oracle.render(th, [CH], [mesh], cam)
    for i in (0, 1, 2):
        th2 = th.copy()
        th2[i] += 2 * math.pi
        np.testing.assert_allclose(oracle.fk(th2, CH), M0, atol=1e-12)
        np.testing.assert_array_equal(oracle.render(th2, [CH], [mesh], cam), m0)


def test_roll_by_pi_symmetry():
    """The instrument is symmetric under a half turn about its shaft (Sec.
    III-A.3): (beta + pi, q1, q2, q3) and (beta, -q1, -q2, q3) give the same
    silhouette up to a few edge pixels from different vertex rounding."""
    wl = scenes.workload("small")
    mesh, cam = wl["mesh"], wl["cam"]
    rng = scenes.rng_for(0, 0)
    for _ in range(3):
        th = scenes.true_pose(rng, cam)
        th_a = th.copy()
        th_a[1] += math.pi
        th_b = th.copy()
        th_b[6], th_b[7] = -th[6], -th[7]          # qhat -> -qhat gives q -> -q for symmetric limits
        a = scenes.words_to_image(oracle.render(th_a, [CH], [mesh], cam), cam.width, cam.height)
        b = scenes.words_to_image(oracle.render(th_b, [CH], [mesh], cam), cam.width, cam.height)
        assert a.sum() > 500
        assert (a ^ b).sum() <= 0.02 * a.sum()


# ------------------------------------------------------------ projection and snapping

def test_optical_axis_projects_to_principal_point():
    cam = scenes.camera(640, 480)
    M = np.zeros((4, 3, 4))
    M[:, :, :3] = np.eye(3)
    M[:, 2, 3] = 0.5                       # everything pushed 0.5 m in front
    mesh = scenes.Mesh(np.array([[0, 0, 0], [0.01, 0, 0], [0, -0.02, 0.5]], np.float32),
                       np.zeros((0, 3), np.int32), np.zeros(3, np.uint8), {})
    uv, sn, fl = oracle.project_snap(M, mesh, cam)
    assert tuple(uv[0]) == (320.0, 240.0)
    assert tuple(sn[0]) == (320 * 256, 240 * 256)
    assert uv[1][0] == pytest.approx(320 + 800 * 0.02)        # x / z * f
    assert uv[2][1] == pytest.approx(240 - 800 * 0.02)
    assert not fl.any()


def test_near_plane_and_guard_band():
    cam = scenes.camera(320, 240, 400.0)
    M = np.zeros((4, 3, 4))
    M[:, :, :3] = np.eye(3)
    verts = np.array([[0, 0, 0.005], [0, 0, -1.0], [1000.0, 0, 0.02], [0, 0, cam.z_near]], np.float32)
    mesh = scenes.Mesh(verts, np.zeros((0, 3), np.int32), np.zeros(4, np.uint8), {})
    uv, sn, fl = oracle.project_snap(M, mesh, cam)
    assert list(fl) == [1, 1, 0, 0]       # z < z_near culled; z == z_near kept
    assert sn[2][0] == 32768 * 256         # clamped to the guard band


def test_snap_rounds_half_to_even():
    cam = scenes.Camera(1.0, 1.0, 0.0, 0.0, 64, 64, 0.01)
    M = np.zeros((4, 3, 4))
    M[:, :, :3] = np.eye(3)
    # u = X / Z with Z = 1: pick X so that 256 u lands on .5 exactly
    xs = np.array([0.5, 1.5, 2.5, -0.5, -1.5]) / 256.0
    verts = np.stack([xs, np.zeros_like(xs), np.ones_like(xs)], 1).astype(np.float32)
    mesh = scenes.Mesh(verts, np.zeros((0, 3), np.int32), np.zeros(len(xs), np.uint8), {})
    _, sn, _ = oracle.project_snap(M, mesh, cam)
    assert list(sn[:, 0]) == [0, 2, 2, 0, -2]


def test_keypoints_project_like_vertices():
    wl = scenes.workload("small")
    cam = wl["cam"]
    th = scenes.true_pose(scenes.rng_for(0, 0), cam)
    M = oracle.fk(th, CH)
    kp = oracle.keypoints(M, CH, cam)
    verts = CH.keypoints[:, :3].astype(np.float32)
    mesh = scenes.Mesh(verts, np.zeros((0, 3), np.int32), CH.keypoints[:, 3].astype(np.uint8), {})
    uv, _, _ = oracle.project_snap(M, mesh, cam)
    np.testing.assert_allclose(kp, uv, rtol=1e-6)   # float32 keypoint storage vs float64
