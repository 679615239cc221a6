"""One-sided rasterisation of closed meshes, pinned on the oracle.

If the triangles of a mesh form a closed, consistently oriented surface
(every directed edge a->b appears as often as b->a), then in the snapped
image plane the triangles with positive signed area cover exactly the pixel
centres that all triangles cover.  The top-left rule is the same as sampling
each centre at an infinitesimally shifted point that lies on no edge, and at
such a point the signed count of covering triangles is the winding number of
the surface's boundary, which is empty: zero.  So a covered centre is covered
by as many positive as negative triangles, at least one of each.  These tests
check the statement on the oracle's own rasteriser (integer edge functions,
top-left rule) from the oracle's snapped vertices, over seeded poses of the
procedural instruments, including vertices clamped to the guard band; and
that it fails for an open mesh, so the closedness condition matters.
"""
import collections

import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_helpers import oracle_snapped


def _closed(tris):
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    c = collections.Counter(map(tuple, e.tolist()))
    return all(c.get((b, a), 0) == n for (a, b), n in c.items())


def _signed_area(sn, tris):
    p = sn.astype(np.int64)
    a, b, c = p[tris[:, 0]], p[tris[:, 1]], p[tris[:, 2]]
    return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])


def _renders(theta, mesh, cam, chain):
    sn, fl = oracle_snapped(theta, chain, mesh, cam)
    assert not fl.any()
    A = _signed_area(sn, mesh.triangles)
    s = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
    full = oracle.raster(s, fl, mesh.triangles, cam.width, cam.height)
    pos = oracle.raster(s, fl, mesh.triangles[A > 0], cam.width, cam.height)
    neg = oracle.raster(s, fl, mesh.triangles[A < 0], cam.width, cam.height)
    return full, pos, neg


@pytest.mark.parametrize("shape", [(32, 28, 3, 1), (64, 150, 6, 4), (100, 170, 7, 5, 1.3, 1.2)])
def test_procedural_meshes_are_closed(shape):
    m = scenes.instrument_mesh(*shape)
    assert _closed(m.triangles)
    assert not _closed(m.triangles[1:])                 # one triangle less: open


def test_one_orientation_renders_the_silhouette_small():
    wl = scenes.workload("small")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    rng = np.random.default_rng(17)
    covered = 0
    for k in range(24):
        th = scenes.true_pose(rng, cam) + 3.0 * scenes.DEFAULT_SCALE * rng.normal(size=9)
        full, pos, neg = _renders(th, mesh, cam, ch)
        assert np.array_equal(full, pos), k
        assert np.array_equal(full, neg), k
        covered += int(oracle.counts(full, full, cam.width, cam.height)[0])
    assert covered > 24 * 500


def test_one_orientation_renders_the_silhouette_track640():
    wl = scenes.workload("track640")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    rng = np.random.default_rng(5)
    for k in range(3):
        th = scenes.true_pose(rng, cam) + scenes.DEFAULT_SCALE * rng.normal(size=9)
        full, pos, neg = _renders(th, mesh, cam, ch)
        assert np.array_equal(full, pos) and np.array_equal(full, neg), k


def test_one_orientation_with_guard_band_clamping():
    """A wide-angle camera close to the shaft: vertices beyond +-32768 px are
    clamped, which moves them but keeps the surface closed."""
    mesh = scenes.instrument_mesh(12, 4, 1, 1)
    ch = scenes.chain()
    cam = scenes.camera(160, 120, f=60000.0)
    rng = np.random.default_rng(2)
    clamped = tried = 0
    while clamped < 8:
        tried += 1
        assert tried < 200
        th = scenes.true_pose(rng, scenes.camera(160, 120)) + scenes.DEFAULT_SCALE * rng.normal(size=9)
        th[5] = 0.05
        sn, fl = oracle_snapped(th, ch, mesh, cam)
        if fl.any() or not (np.abs(sn) >= 256 * 32768).any():
            continue                                   # keep poses in front of the near plane that clamp
        clamped += 1
        full, pos, neg = _renders(th, mesh, cam, ch)
        assert np.array_equal(full, pos) and np.array_equal(full, neg), tried


def test_open_mesh_is_not_one_sided():
    """Without the end discs the shaft is an open tube: seen along its axis,
    its inside shows through the open end and is covered by triangles of one
    orientation only."""
    mesh = scenes.instrument_mesh(32, 28, 3, 1)
    s = 32
    side = 2 * s * 29
    keep = np.ones(mesh.n_triangles, dtype=bool)
    keep[side:side + 2 * s] = False                     # the two end discs of the shaft
    assert _closed(mesh.triangles) and not _closed(mesh.triangles[keep])
    cam = scenes.camera(320, 240, 400.0)
    ch = scenes.chain()
    # shaft pointing away from the camera, nearly along the optical axis
    th = np.array([np.pi - 0.05, 0.0, 0.05, 0.0, 0.0, 0.08, 0.0, 0.0, 0.5])
    sn, fl = oracle_snapped(th, ch, mesh, cam)
    tris = mesh.triangles[keep]
    A = _signed_area(sn, tris)
    s32 = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
    full = oracle.raster(s32, fl, tris, cam.width, cam.height)
    pos = oracle.raster(s32, fl, tris[A > 0], cam.width, cam.height)
    neg = oracle.raster(s32, fl, tris[A < 0], cam.width, cam.height)
    assert not (np.array_equal(full, pos) and np.array_equal(full, neg))
