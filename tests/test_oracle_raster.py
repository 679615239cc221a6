"""Pins of the oracle rasteriser (the renderer R of Sec. III-A.2, S in {0,1}^{HxW}).

Closed-form pixel counts (unit square, s x s squares, right triangles), the
no-double-coverage property of shared edges, exact integer translation,
winding independence, culling rules, and agreement with an independent exact
rational brute force (oracle/brute.py) on random tiny scenes.
"""
import numpy as np
import pytest

import oracle
import scenes
from oracle import brute

Q = 256  # subpixel units per pixel


def _raster(verts_px, tris, W, H, flags=None, counts=True):
    sn = np.rint(np.asarray(verts_px, dtype=np.float64) * Q).astype(np.int32)
    fl = np.zeros(len(sn), np.uint8) if flags is None else np.asarray(flags, np.uint8)
    return oracle.raster(sn, fl, np.asarray(tris, np.int32), W, H, with_counts=counts)


def _img(words, W, H):
    return scenes.words_to_image(words, W, H)


def test_unit_pixel_square_gives_one():
    for (x, y) in [(3, 4), (0, 0), (15, 11)]:
        v = [(x, y), (x + 1, y), (x + 1, y + 1), (x, y + 1)]
        m, c = _raster(v, [(0, 1, 2), (0, 2, 3)], 16, 12)
        img = _img(m, 16, 12)
        assert img.sum() == 1 and img[y, x]
        assert c.max() == 1


@pytest.mark.parametrize("s", [1, 2, 5, 8, 13])
@pytest.mark.parametrize("offset", [0.0, 0.5])   # corners on pixel corners / on pixel centres
def test_square_gives_s_squared(s, offset):
    x0, y0 = 3 + offset, 2 + offset
    v = [(x0, y0), (x0 + s, y0), (x0 + s, y0 + s), (x0, y0 + s)]
    for tris in ([(0, 1, 2), (0, 2, 3)], [(0, 1, 3), (1, 2, 3)], [(0, 2, 1), (0, 3, 2)]):
        m, c = _raster(v, tris, 32, 24)
        assert _img(m, 32, 24).sum() == s * s
        assert c.sum() == s * s              # the diagonal is owned by exactly one triangle


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_right_triangle_and_complement(n):
    W = H = 20
    a, cmp_ = [(0, 0), (n, 0), (0, n)], [(n, 0), (n, n), (0, n)]
    ma, ca = _raster(a, [(0, 1, 2)], W, H)
    mb, cb = _raster(cmp_, [(0, 1, 2)], W, H)
    assert _img(ma, W, H).sum() == n * (n - 1) // 2     # centres on the hypotenuse excluded
    assert _img(mb, W, H).sum() == n * (n + 1) // 2     # ... and owned by the complement
    assert ((ca + cb) == 1).sum() == n * n and (ca + cb).max() == 1


def test_watertight_jittered_grid():
    rng = np.random.default_rng(5)
    W, H = 48, 40
    nx, ny = 7, 6
    gx = np.linspace(2.0, 45.0, nx + 1)
    gy = np.linspace(1.5, 37.0, ny + 1)
    P = np.stack(np.meshgrid(gx, gy, indexing="ij"), -1)
    P[1:-1, 1:-1] += rng.uniform(-1.0, 1.0, size=P[1:-1, 1:-1].shape)
    # snap some interior vertices exactly onto pixel centres to exercise ties
    P[2, 2] = [np.floor(P[2, 2, 0]) + 0.5, np.floor(P[2, 2, 1]) + 0.5]
    P[4, 3] = [np.floor(P[4, 3, 0]) + 0.5, np.floor(P[4, 3, 1]) + 0.5]
    verts = P.reshape(-1, 2)
    idx = np.arange((nx + 1) * (ny + 1)).reshape(nx + 1, ny + 1)
    tris = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = idx[i, j], idx[i + 1, j], idx[i + 1, j + 1], idx[i, j + 1]
            if rng.random() < 0.5:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
            if rng.random() < 0.3:           # random winding flips
                tris[-1] = tris[-1][::-1]
    m, c = _raster(verts, tris, W, H)
    assert c.max() == 1
    # the union equals the grid's outer rectangle rule: x in [2, 45), y in [1.5, 37) centres
    xs = np.arange(W) + 0.5
    ys = np.arange(H) + 0.5
    inside = (ys[:, None] >= 1.5) & (ys[:, None] < 37.0) & (xs[None, :] >= 2.0) & (xs[None, :] < 45.0)
    np.testing.assert_array_equal(_img(m, W, H), inside)


def test_integer_shift_shifts_mask():
    rng = np.random.default_rng(6)
    W, H = 64, 48
    v = rng.uniform(5, 30, size=(30, 2))
    tris = rng.integers(0, 30, size=(25, 3))
    sn = np.rint(v * Q).astype(np.int32)
    fl = np.zeros(30, np.uint8)
    base = _img(oracle.raster(sn, fl, tris, W, H), W, H)
    for k, l in [(1, 0), (0, 3), (7, 5), (13, 2)]:
        sh = sn + np.array([k * Q, l * Q], np.int32)
        moved = _img(oracle.raster(sh, fl, tris, W, H), W, H)
        np.testing.assert_array_equal(moved[l:, k:], base[:H - l, :W - k])
        assert moved[:l].sum() == 0 and moved[:, :k].sum() == 0


def test_vertex_order_does_not_matter():
    rng = np.random.default_rng(7)
    W, H = 40, 30
    v = rng.uniform(-5, 45, size=(40, 2))
    tris = rng.integers(0, 40, size=(60, 3))
    sn = np.rint(v * Q).astype(np.int32)
    fl = np.zeros(40, np.uint8)
    ref, cref = oracle.raster(sn, fl, tris, W, H, with_counts=True)
    for perm in [(1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)]:
        m, c = oracle.raster(sn, fl, tris[:, perm], W, H, with_counts=True)
        np.testing.assert_array_equal(m, ref)
        np.testing.assert_array_equal(c, cref)


def test_culling_rules():
    W, H = 16, 16
    v = [(1, 1), (9, 1), (1, 9), (20, 20), (30, 20), (20, 30), (2, 2), (4, 4), (6, 6)]
    tris = [(0, 1, 2), (3, 4, 5), (6, 7, 8)]
    # second triangle fully off-screen, third degenerate (collinear)
    m = _raster(v, tris, W, H, counts=False)
    only_first = _raster(v[:3], [(0, 1, 2)], W, H, counts=False)
    np.testing.assert_array_equal(m, only_first)
    # a flagged (behind near plane) vertex drops every triangle that uses it
    m2 = _raster(v, tris, W, H, flags=[0, 1, 0, 0, 0, 0, 0, 0, 0], counts=False)
    assert _img(m2, W, H).sum() == 0


@pytest.mark.parametrize("W,H", [(13, 11), (8, 8), (17, 9)])
def test_padding_bits_stay_zero(W, H):
    v = [(-10, -10), (40, -10), (-10, 40)]
    m = _raster(v, [(0, 1, 2)], W, H, counts=False)
    img = _img(m, W, H)
    assert img.all()
    full = scenes.words_to_image(m, ((W + 7) // 8) * 8, ((H + 7) // 8) * 8)
    assert full.sum() == W * H


def test_large_guard_band_triangle_exact():
    """A triangle with vertices far outside the screen (int64 edge functions)
    covers exactly the half plane it cuts through the image."""
    W, H = 32, 24
    big = 30000.0
    # edge from (-big, 10.5) to (big, 10.5): triangle above (y < 10.5) in y-down coordinates
    v = [(-big, 10.5), (big, 10.5), (0.0, -big)]
    m = _raster(v, [(0, 1, 2)], W, H, counts=False)
    img = _img(m, W, H)
    # centres with y + 0.5 < 10.5 are strictly inside; y + 0.5 == 10.5 lies on the bottom edge (excluded)
    assert img[:10].all() and not img[10:].any()


def test_oracle_matches_rational_brute_force():
    rng = np.random.default_rng(8)
    for case in range(12):
        W, H = int(rng.integers(5, 14)), int(rng.integers(5, 14))
        nv = 12
        # mix free positions with positions on pixel centres / corners to exercise ties
        v = rng.uniform(-3, max(W, H) + 3, size=(nv, 2))
        k = rng.random(nv)
        v[k < 0.3] = np.floor(v[k < 0.3]) + 0.5
        v[(k >= 0.3) & (k < 0.5)] = np.floor(v[(k >= 0.3) & (k < 0.5)])
        sn = np.rint(v * Q).astype(np.int32)
        fl = (rng.random(nv) < 0.08).astype(np.uint8)
        tris = rng.integers(0, nv, size=(10, 3))
        _, c = oracle.raster(sn, fl, tris, W, H, with_counts=True)
        b = np.array(brute.coverage_counts(sn, fl, tris, W, H))
        np.testing.assert_array_equal(c, b, err_msg=f"case {case}")
