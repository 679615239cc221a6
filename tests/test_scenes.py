"""Sanity of the seeded input generators (data only)."""
import numpy as np

import scenes


def test_mesh_triangle_counts():
    # shaft sides 2 s (r + 1) and end discs 2 s, box 12 k^2, jaws 16 m^2
    m = scenes.instrument_mesh(32, 28, 3, 1)
    assert m.n_triangles == 2 * 32 * 29 + 2 * 32 + 12 * 9 + 16 == 2044
    m2 = scenes.instrument_mesh(64, 150, 6, 4)
    assert m2.n_triangles == 2 * 64 * 151 + 2 * 64 + 12 * 36 + 16 * 16 == 20144
    # welded face grids: shaft rings + 2 disc centres, box surface grid, jaw prisms
    assert m.n_vertices == 32 * 30 + 2 + (6 * 3 * 3 + 2) + 2 * 6
    for mesh in (m, m2, scenes.mesh_for_triangles(35000, 1.3, 1.2), scenes.mesh_for_triangles(3000)):
        assert mesh.triangles.min() >= 0 and mesh.triangles.max() < mesh.n_vertices
        assert np.all(np.diff(mesh.vertex_link.astype(int)) >= 0)       # sorted by link
        assert set(np.unique(mesh.vertex_link)) == {0, 1, 2, 3}
        assert mesh.vertices.dtype == np.float32 and mesh.triangles.dtype == np.int32
        # every triangle uses vertices of a single link
        tl = mesh.vertex_link[mesh.triangles]
        assert np.all(tl.min(1) == tl.max(1))
    assert abs(scenes.mesh_for_triangles(35000).n_triangles - 35000) < 200


def test_mask_layout_roundtrip():
    rng = np.random.default_rng(0)
    for W, H in [(320, 240), (13, 9), (960, 540)]:
        img = rng.random((H, W)) < 0.5
        w = scenes.image_to_words(img)
        assert w.shape == ((H + 7) // 8, (W + 7) // 8)
        np.testing.assert_array_equal(scenes.words_to_image(w, W, H), img)
    # bit (y%8)*8 + x%8 of word [y/8][x/8]
    img = np.zeros((16, 16), bool)
    img[9, 3] = True
    w = scenes.image_to_words(img)
    assert w[1, 0] == np.uint64(1) << np.uint64(8 + 3)


def test_flips_distinct_and_exact_count():
    idx = scenes.flip_indices(scenes.rng_for(1, scenes.SUB_FLIPS), 640, 480)
    assert len(idx) == 3072 and len(np.unique(idx)) == 3072
    w = np.zeros((60, 80), np.uint64)
    f = scenes.apply_flips(w, 640, 480, idx)
    assert scenes.words_to_image(f, 640, 480).sum() == 3072


def test_true_pose_ranges_and_determinism():
    cam = scenes.camera(640, 480)
    a = scenes.true_pose(scenes.rng_for(1, 0), cam)
    b = scenes.true_pose(scenes.rng_for(1, 0), cam)
    assert np.array_equal(a, b)
    assert 0.08 <= a[5] <= 0.15


def test_trajectory_steps():
    cam = scenes.camera(640, 480)
    tr = scenes.trajectory(scenes.rng_for(1, scenes.SUB_TRAJ), cam, 100)
    assert tr.shape == (100, 9)
    dt = np.linalg.norm(np.diff(tr[:, 3:6], axis=0), axis=1)
    np.testing.assert_allclose(dt, 0.001, rtol=1e-9)


def test_occluder_covers_requested_fraction():
    img = np.zeros((100, 120), bool)
    img[20:60, 30:100] = True
    rect, phi = scenes.occluder_rect(img, np.random.default_rng(3))
    x0, y0, x1, y1 = rect
    frac = img[y0:y1, x0:x1].sum() / img.sum()
    assert 0.1 <= phi <= 0.3 and frac >= phi
    assert scenes.apply_occluder(img, rect).sum() == img.sum() - img[y0:y1, x0:x1].sum()


def test_hermite_trajectory_is_seeded_bounded_and_smooth():
    cam = scenes.camera(700, 493)
    a = scenes.hermite_trajectory(scenes.rng_for(5, scenes.SUB_TRAJ), cam, 300)
    b = scenes.hermite_trajectory(scenes.rng_for(5, scenes.SUB_TRAJ), cam, 300)
    assert np.array_equal(a, b) and a.shape == (300, 9)
    assert a[:, 5].min() > 0.07 and a[:, 5].max() < 0.16          # depth band (plus the OU noise)
    d2 = np.abs(np.diff(a, 2, axis=0))
    assert d2[:, 3:6].max() < 2e-3 and d2[:, 0:3].max() < 0.02      # no jumps after the low-pass


def test_perturb_mask_only_changes_pixels_near_the_boundary():
    from scipy import ndimage
    img = np.zeros((120, 160), bool)
    img[30:90, 40:120] = True
    for seed in range(8):
        out = scenes.perturb_mask(np.random.default_rng(seed), img)
        changed = out ^ img
        near = ndimage.binary_dilation(img ^ ndimage.binary_erosion(img), iterations=8)
        assert not np.any(changed & ~near), seed
