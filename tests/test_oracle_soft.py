"""Pins of the soft-silhouette oracle and of the forward-kinematics Jacobian.

- The Jacobian equals central differences of the oracle's forward kinematics.
- An isolated triangle in the image plane: along a pixel column near one leg
  the signed distance is known from the geometry (py - 8 inside, py - 8
  outside as well), so S is the shifted logistic of it, exactly.
- Two triangles: S is the probabilistic OR of the two single-triangle images.
- As sigma -> 0, S > 0.5 reproduces the integer rasteriser's hard mask except
  at pixels next to an edge of the hard mask.
- The analytic gradient equals FP64 central differences (h = 1e-4 in the
  normalised coordinates), for one arm and for two arms.
"""
import math

import numpy as np
import pytest

import oracle
import scenes

S0 = 1.0 / (1.0 + math.exp(10.0))


def shifted(d, sigma):
    if d < -10.0 * sigma:
        return 0.0
    s = 1.0 / (1.0 + math.exp(-d / sigma))
    return (s - S0) / (1.0 - S0)


def plane_mesh(tris_uv, f=128.0):
    """Triangles given in pixels, placed in the plane z = 1 m of the camera
    (identity pose, shaft link): u = f X + 0 with X = u / f exact in float32."""
    v = []
    for tri in tris_uv:
        for (u, w) in tri:
            v.append((u / f, w / f, 0.0))
    V = np.array(v, dtype=np.float32)
    T = np.arange(len(v), dtype=np.int32).reshape(-1, 3)
    return scenes.Mesh(V, T, np.zeros(len(v), dtype=np.uint8), {})


def plane_setup(tris_uv, W=64, H=64):
    cam = scenes.Camera(128.0, 128.0, 0.0, 0.0, W, H)
    theta = np.array([0, 0, 0, 0, 0, 1.0, 0, 0, 0.5])
    return cam, theta, plane_mesh(tris_uv)


def test_fk_jacobian_matches_central_differences():
    rng = np.random.default_rng(5)
    for jaw in (1.0, 1.3):
        ch = scenes.chain(jaw)
        for _ in range(4):
            th = np.concatenate([rng.uniform(-2, 2, 3), rng.uniform(-0.1, 0.1, 3), rng.uniform(-1.5, 1.5, 3)])
            J = oracle.fk_jacobian(th, ch)
            h = 1e-6
            for k in range(9):
                e = np.zeros(9)
                e[k] = h
                fd = (oracle.fk(th + e, ch) - oracle.fk(th - e, ch)).reshape(4, 12) / (2 * h)
                np.testing.assert_allclose(J[k], fd, atol=2e-8, err_msg=f"parameter {k}")


@pytest.mark.parametrize("sigma", [1.0, 0.6])
def test_isolated_triangle_is_the_shifted_logistic_of_the_distance(sigma):
    cam, theta, mesh = plane_setup([[(8.0, 8.0), (56.0, 8.0), (8.0, 56.0)]])
    _, S, _ = oracle.soft(theta, [scenes.chain()], [mesh], cam, sigma, want_S=True)
    # column px = 20.5: for py < 20.5 the leg v = 8 is the nearest edge (the
    # other leg is 12.5 px away, the hypotenuse farther), inside and outside
    for y in range(0, 20):
        py = y + 0.5
        assert S[y, 20] == pytest.approx(shifted(py - 8.0, sigma), abs=1e-14), y
    # far from the triangle nothing is drawn; deep inside S -> 1
    assert S[63, 63] == 0.0 and S[0, 63] == 0.0
    assert S[20, 20] > 1.0 - 1e-5


def test_two_triangles_combine_by_probabilistic_or():
    a = [(8.0, 8.0), (30.0, 8.0), (8.0, 30.0)]
    b = [(8.0, 36.0), (30.0, 36.0), (8.0, 58.0)]
    cam, theta, ma = plane_setup([a])
    _, Sa, _ = oracle.soft(theta, [scenes.chain()], [ma], cam, 1.0, want_S=True)
    _, Sb, _ = oracle.soft(theta, [scenes.chain()], [plane_mesh([b])], cam, 1.0, want_S=True)
    _, Sab, _ = oracle.soft(theta, [scenes.chain()], [plane_mesh([a, b])], cam, 1.0, want_S=True)
    np.testing.assert_allclose(Sab, 1.0 - (1.0 - Sa) * (1.0 - Sb), atol=1e-15)
    assert np.sum((Sa > 1e-6) & (Sb > 1e-6)) > 20          # the bands do overlap


def test_small_sigma_reproduces_the_hard_mask_away_from_edges():
    wl = scenes.workload("small")
    cam, mesh, ch = wl["cam"], wl["mesh"], scenes.chain()
    rng = scenes.rng_for(0, scenes.SUB_POSE)
    th = scenes.true_pose(rng, cam)
    _, S, _ = oracle.soft(th, [ch], [mesh], cam, 0.01, want_S=True)
    hard = scenes.words_to_image(oracle.render(th, [ch], [mesh], cam), cam.width, cam.height)
    soft = S > 0.5
    diff = soft != hard
    # a differing pixel must touch a change of the hard mask (an edge)
    pad = np.pad(hard, 1, mode="edge")
    edge = np.zeros_like(hard)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            edge |= pad[1 + dy:1 + dy + hard.shape[0], 1 + dx:1 + dx + hard.shape[1]] != hard
    assert hard.sum() > 500
    assert not np.any(diff & ~edge)
    assert diff.sum() < 0.02 * hard.sum()


def _fd_check(thetas, chains, meshes, cam, target, scale, sigma=1.0):
    L0, _, g = oracle.soft(thetas, chains, meshes, cam, sigma, target, want_grad=True)
    h = 1e-4
    fd = np.zeros_like(g)
    for k in range(g.size):
        e = np.zeros(g.size)
        e[k] = h * scale[k]                # step of h in the normalised coordinate
        lp = oracle.soft(thetas + e, chains, meshes, cam, sigma, target)[0]
        lm = oracle.soft(thetas - e, chains, meshes, cam, sigma, target)[0]
        fd[k] = (lp - lm) / (2 * h)
    gx = g * scale                          # gradient in the normalised coordinates
    rel = np.linalg.norm(gx - fd) / np.linalg.norm(fd)
    assert L0 > 0 and np.linalg.norm(fd) > 0
    assert rel <= 1e-3, (rel, gx, fd)
    return gx, fd


def test_gradient_matches_central_differences_one_arm():
    cam = scenes.camera(160, 120, 200.0)
    mesh, ch = scenes.instrument_mesh(24, 16, 2, 1), scenes.chain()
    rng = scenes.rng_for(0, scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    target = oracle.render(truth, [ch], [mesh], cam)
    th = truth + scenes.DEFAULT_SCALE * rng.normal(size=9) * 0.5
    _fd_check(th, [ch], [mesh], cam, target, scenes.DEFAULT_SCALE)


def test_gradient_matches_central_differences_two_arms():
    cam = scenes.camera(160, 120, 200.0)
    meshes = [scenes.instrument_mesh(16, 12, 2, 1), scenes.instrument_mesh(20, 12, 2, 1, jaw_scale=1.3)]
    chains = [scenes.chain(), scenes.chain(1.3)]
    rng = scenes.rng_for(1, scenes.SUB_POSE)
    truth = np.concatenate([scenes.true_pose(rng, cam) for _ in range(2)])
    target = oracle.render(truth, chains, meshes, cam)
    th = truth + np.tile(scenes.DEFAULT_SCALE, 2) * rng.normal(size=18) * 0.5
    _fd_check(th, chains, meshes, cam, target, np.tile(scenes.DEFAULT_SCALE, 2))


# ---------------------------------------------------------------- face-major form

def _banded_vs_literal(theta, chains, meshes, cam, sigma, target):
    L1, S1, g1 = oracle.soft(theta, chains, meshes, cam, sigma, target, want_S=True, want_grad=True)
    L2, S2, g2 = oracle.soft(theta, chains, meshes, cam, sigma, target, want_S=True, want_grad=True, banded=True)
    return L1, S1, g1, L2, S2, g2


@pytest.mark.parametrize("sigma", [1.0, 0.7])
def test_banded_form_equals_the_literal_one(sigma):
    """Face-major over each face's 10-sigma box: S and the loss are the same
    numbers, the gradient the same to rounding (one and two arms)."""
    rng = np.random.default_rng(21)
    cam = scenes.camera(96, 72, f=110.0)
    meshes = [scenes.instrument_mesh(12, 4, 1, 1), scenes.instrument_mesh(10, 3, 1, 1, jaw_scale=1.3)]
    chains = [scenes.chain(), scenes.chain(1.3)]
    for n_arms in (1, 2):
        for _ in range(3):
            th = np.concatenate([scenes.true_pose(rng, cam) for _ in range(n_arms)])
            target = oracle.render(th + 0.3 * np.tile(scenes.DEFAULT_SCALE, n_arms), chains[:n_arms],
                                   meshes[:n_arms], cam)
            L1, S1, g1, L2, S2, g2 = _banded_vs_literal(th, chains[:n_arms], meshes[:n_arms], cam, sigma, target)
            assert L1 == L2 and np.array_equal(S1, S2)
            assert L1 > 0 and np.linalg.norm(g1) > 0
            assert np.linalg.norm(g2 - g1) <= 1e-12 * np.linalg.norm(g1)


def test_banded_form_with_factors_exactly_zero():
    """Deep inside large faces the logistic is 1 in FP64 and the factor 1 - prob
    is exactly zero: the product over the other faces must still follow the
    definition (zero whenever another factor is zero)."""
    cam, theta, mesh = plane_setup([[(4, 4), (60, 6), (8, 58)], [(10, 12), (58, 40), (30, 60)],
                                    [(2, 30), (40, 2), (50, 50)]])
    target = np.zeros(((cam.height + 7) // 8, (cam.width + 7) // 8), np.uint64)
    target[2:5, 2:5] = np.uint64(0xFFFFFFFFFFFFFFFF)
    for sigma in (0.25, 0.5):
        L1, S1, g1, L2, S2, g2 = _banded_vs_literal(theta, [scenes.chain()], [mesh], cam, sigma, target)
        assert (S1 == 1.0).sum() > 100            # factors exactly zero occur
        assert L1 == L2 and np.array_equal(S1, S2)
        assert np.linalg.norm(g2 - g1) <= 1e-12 * max(np.linalg.norm(g1), 1e-300)


def _fd_job(args):
    th, k, h, scale = args
    wl = scenes.workload("soft640")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    truth = scenes.true_pose(scenes.rng_for(wl["index"], scenes.SUB_POSE), cam)
    target = oracle.render(truth, [ch], [mesh], cam)
    e = np.zeros(9)
    e[k] = h * scale[k]
    lp, _, _ = oracle.soft(th + e, [ch], [mesh], cam, 1.0, target, banded=True)
    lm, _, _ = oracle.soft(th - e, [ch], [mesh], cam, 1.0, target, banded=True)
    return (lp - lm) / (2.0 * h * scale[k])


@pytest.mark.slow
def test_banded_gradient_matches_central_differences_at_full_size():
    """The 49744-triangle instrument at 640x480, sigma = 1 px: the analytic
    gradient of 16 seeded candidates equals central differences (h = 1e-4 in
    the normalised coordinates) to 1e-3 relative, norm-wise."""
    import multiprocessing as mp
    wl = scenes.workload("soft640")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    rng = scenes.rng_for(wl["index"], scenes.SUB_POSE)
    truth = scenes.true_pose(rng, cam)
    target = oracle.render(truth, [ch], [mesh], cam)
    cands = [truth + scenes.DEFAULT_SCALE * rng.normal(size=9) for _ in range(16)]
    jobs = [(th, k, 1e-4, scenes.DEFAULT_SCALE) for th in cands for k in range(9)]
    with mp.get_context("fork").Pool(min(8, mp.cpu_count())) as pool:
        fd = np.array(pool.map(_fd_job, jobs)).reshape(16, 9)
    for c, th in enumerate(cands):
        _, _, g = oracle.soft(th, [ch], [mesh], cam, 1.0, target, want_grad=True, banded=True)
        assert np.linalg.norm(g) > 0
        assert np.linalg.norm(fd[c] - g) <= 1e-3 * np.linalg.norm(g), c
