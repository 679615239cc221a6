"""Host-side mesh planning for the one-sided raster path (no device call).

* tk_mesh_closed against its definition computed here: every directed edge
  a->b occurs as often as b->a (edges of a repeated vertex ignored).
* tk_mesh_plane_order is a permutation of the triangles that renders the same
  silhouette, and groups them so that, in seeded poses, most 64-triangle
  chunks of the order the device mesh uses (plane order, then claim order) are
  wholly of one orientation in the snapped image plane (the chunks the
  rasteriser can skip or keep whole).
"""
import collections
import os

import numpy as np
import pytest

import oracle
import scenes
from tests.gpu_helpers import oracle_snapped

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_11404_amd", "libtk.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")


def closed_by_definition(tris):
    c = collections.Counter()
    for t in np.asarray(tris).tolist():
        for e in range(3):
            a, b = t[e], t[(e + 1) % 3]
            if a != b:
                c[(a, b)] += 1
    return all(c.get((b, a), 0) == n for (a, b), n in c.items())


def test_closed_matches_its_definition():
    from paper_2603_11404_amd import tk
    rng = np.random.default_rng(1)
    cases = []
    for shape in [(32, 28, 3, 1), (12, 4, 1, 1), (64, 150, 6, 4)]:
        t = scenes.instrument_mesh(*shape).triangles
        cases.append((t, True))
        cases.append((t[1:], False))                                   # a hole
        flipped = t.copy()
        flipped[7] = flipped[7][::-1]
        cases.append((flipped, False))                                 # one triangle wound the other way
        cases.append((np.concatenate([t, t[:1][:, ::-1]]), False))     # a dangling two-sided triangle... open
        cases.append((np.concatenate([t, t[:1], t[:1][:, [0, 2, 1]]]), True))   # ...and its pair: closed
        perm = rng.permutation(len(t))
        cases.append((t[perm], True))                                  # order does not matter
    degenerate = np.array([[0, 1, 2], [0, 2, 1], [3, 3, 4]], np.int32)
    cases.append((degenerate, True))
    cases.append((np.zeros((0, 3), np.int32), True))
    for t, want in cases:
        n_v = int(t.max()) + 1 if t.size else 1
        assert closed_by_definition(t) == want
        assert tk.mesh_closed(t, n_v) == want


def test_closed_argument_errors():
    from paper_2603_11404_amd import tk
    import ctypes
    L = tk.lib()
    t = np.array([[0, 1, 5]], np.int32)
    out = ctypes.c_int32(-7)
    assert L.tk_mesh_closed(t.ctypes.data, 1, 5, ctypes.byref(out)) == tk.TK_ERR_INVALID_ARGUMENT
    assert L.tk_mesh_closed(t.ctypes.data, 1, 6, None) == tk.TK_ERR_INVALID_ARGUMENT
    assert L.tk_mesh_closed(None, 1, 6, ctypes.byref(out)) == tk.TK_ERR_INVALID_ARGUMENT
    assert out.value == -7


def test_plane_order_is_a_permutation_that_renders_the_same():
    from paper_2603_11404_amd import tk
    wl = scenes.workload("small")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    out = tk.mesh_plane_order(mesh.vertices, mesh.vertex_link, mesh.triangles)
    assert out.dtype == np.int32 and out.shape == mesh.triangles.shape
    assert sorted(map(tuple, out)) == sorted(map(tuple, mesh.triangles))
    assert not np.array_equal(out, mesh.triangles)
    # links stay in their order; within a link, triangles of one plane are contiguous
    links = mesh.vertex_link[out[:, 0]]
    assert np.all(np.diff(links.astype(int)) >= 0)
    rng = scenes.rng_for(3, scenes.SUB_POSE)
    for _ in range(3):
        th = scenes.true_pose(rng, cam)
        sn, fl = oracle_snapped(th, ch, mesh, cam)
        s = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
        a = oracle.raster(s, fl, mesh.triangles, cam.width, cam.height)
        assert a.any() and np.array_equal(a, oracle.raster(s, fl, out, cam.width, cam.height))


@pytest.mark.parametrize("name", ["small", "track640"])
def test_device_order_chunks_are_mostly_of_one_orientation(name):
    from paper_2603_11404_amd import tk
    wl = scenes.workload(name)
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    order = tk.mesh_chunk_order(mesh.vertices, tk.mesh_plane_order(mesh.vertices, mesh.vertex_link,
                                                                   mesh.triangles))
    rng = np.random.default_rng(4)
    uniform = total = 0
    for _ in range(4):
        th = scenes.true_pose(rng, cam) + scenes.DEFAULT_SCALE * rng.normal(size=9)
        sn, fl = oracle_snapped(th, ch, mesh, cam)
        p = sn.astype(np.int64)
        a, b, c = p[order[:, 0]], p[order[:, 1]], p[order[:, 2]]
        pos = ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])) > 0
        for k in range(0, len(order), 64):
            blk = pos[k:k + 64]
            uniform += int(blk.all() or not blk.any())
            total += 1
    assert uniform >= 0.85 * total, (uniform, total)


def test_plane_order_argument_errors():
    from paper_2603_11404_amd import tk
    L = tk.lib()
    m = scenes.instrument_mesh(12, 4, 1, 1)
    v = np.ascontiguousarray(m.vertices)
    lk = np.ascontiguousarray(m.vertex_link)
    t = np.ascontiguousarray(m.triangles)
    out = np.full_like(t, -7)
    bad = t.copy()
    bad[3, 1] = m.n_vertices
    for args in [(v.ctypes.data, lk.ctypes.data, m.n_vertices, bad.ctypes.data, len(t), out.ctypes.data),
                 (None, lk.ctypes.data, m.n_vertices, t.ctypes.data, len(t), out.ctypes.data),
                 (v.ctypes.data, None, m.n_vertices, t.ctypes.data, len(t), out.ctypes.data),
                 (v.ctypes.data, lk.ctypes.data, m.n_vertices, t.ctypes.data, len(t), t.ctypes.data)]:
        assert L.tk_mesh_plane_order(*args) == tk.TK_ERR_INVALID_ARGUMENT
    assert np.all(out == -7)
