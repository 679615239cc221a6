"""tk_mesh_chunk_order, the host-side claim order of a mesh's triangles for
the raster kernels (no device call: runs without a GPU).

The silhouette S of Sec. III-A.2 is an OR over triangles, so a reordered
triangle list must render the same mask; the tests check that on the oracle,
and the block order against its definition computed here in numpy."""
import os

import numpy as np
import pytest

import oracle
import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_11404_amd", "libtk.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libtk.so not built")


def expected_order(vertices, tris):
    """Blocks of 64 cut from the end, full blocks by decreasing summed area
    (ties in list order), the short block of the first T mod 64 last."""
    T = tris.shape[0]
    head = T % 64
    P = np.asarray(vertices, np.float64)[tris]
    area2 = np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    full = (T - head) // 64
    cost = np.array([area2[head + 64 * k: head + 64 * (k + 1)].sum() for k in range(full)])
    order = np.argsort(-cost, kind="stable")
    parts = [tris[head + 64 * k: head + 64 * (k + 1)] for k in order] + [tris[:head]]
    return np.concatenate(parts) if parts else tris[:0]


def random_mesh(rng, V, T):
    verts = rng.normal(size=(V, 3)).astype(np.float32) * rng.uniform(0.001, 0.05, size=(V, 1)).astype(np.float32)
    tris = rng.integers(0, V, size=(T, 3)).astype(np.int32)
    return verts, tris


@pytest.mark.parametrize("T", [0, 1, 63, 64, 65, 128, 64 * 37 + 21])
def test_block_order_matches_its_definition(T):
    from paper_2603_11404_amd import tk
    rng = np.random.default_rng(T + 11)
    verts, tris = random_mesh(rng, 300, T)
    out = tk.mesh_chunk_order(verts, tris)
    assert out.shape == tris.shape and out.dtype == np.int32
    np.testing.assert_array_equal(out, expected_order(verts, tris))
    # a permutation of the rows, whole blocks kept together, costs non-increasing
    assert sorted(map(tuple, out)) == sorted(map(tuple, tris))
    head = T % 64
    np.testing.assert_array_equal(out[T - head:], tris[:head])
    P = verts.astype(np.float64)[out]
    a2 = np.linalg.norm(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]), axis=1)
    blocks = [a2[64 * k: 64 * (k + 1)].sum() for k in range((T - head) // 64)]
    assert all(x >= y for x, y in zip(blocks, blocks[1:]))


def test_instrument_mesh_renders_the_same_silhouette():
    from paper_2603_11404_amd import tk
    wl = scenes.workload("small")
    mesh, cam, ch = wl["mesh"], wl["cam"], scenes.chain()
    out = tk.mesh_chunk_order(mesh.vertices, mesh.triangles)
    assert not np.array_equal(out, mesh.triangles)   # the order does change on this mesh
    rng = scenes.rng_for(3, scenes.SUB_POSE)
    for _ in range(3):
        th = scenes.true_pose(rng, cam)
        M = oracle.fk(th, ch)
        _, sn, fl = oracle.project_snap(M, mesh, cam)
        a = oracle.raster(sn, fl, mesh.triangles, cam.width, cam.height)
        b = oracle.raster(sn, fl, out, cam.width, cam.height)
        assert a.any()
        np.testing.assert_array_equal(a, b)


def test_argument_errors_leave_the_output_untouched():
    from paper_2603_11404_amd import tk
    L = tk.lib()
    verts, tris = random_mesh(np.random.default_rng(5), 40, 100)
    out = np.full_like(tris, -7)
    bad = tris.copy()
    bad[57, 2] = 40   # one past the last vertex
    for args in [(verts.ctypes.data, 40, bad.ctypes.data, 100, out.ctypes.data),
                 (verts.ctypes.data, 0, tris.ctypes.data, 100, out.ctypes.data),
                 (verts.ctypes.data, 40, tris.ctypes.data, -1, out.ctypes.data),
                 (None, 40, tris.ctypes.data, 100, out.ctypes.data),
                 (verts.ctypes.data, 40, tris.ctypes.data, 100, None),
                 (verts.ctypes.data, 40, tris.ctypes.data, 100, tris.ctypes.data)]:
        assert L.tk_mesh_chunk_order(*args) == tk.TK_ERR_INVALID_ARGUMENT
        assert len(L.tk_last_error()) > 0
    assert np.all(out == -7)
    # overlapping by one row
    buf = np.concatenate([tris, tris[:1]])
    assert L.tk_mesh_chunk_order(verts.ctypes.data, 40, buf.ctypes.data, 100, buf[1:].ctypes.data) == \
        tk.TK_ERR_INVALID_ARGUMENT
    # no triangles: nothing to do, NULL arrays accepted
    assert L.tk_mesh_chunk_order(verts.ctypes.data, 40, None, 0, None) == tk.TK_OK
