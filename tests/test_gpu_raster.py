"""GPU parity of the raster and count kernels against the CPU oracle.

Masks and integer counts must be bit-exact given the same snapped vertices;
the snapped vertices fed to both sides come from the oracle's FP64 projection
or from synthetic seeded coordinates, never from the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from tests.gpu_helpers import (INT32_MIN, candidates, i64_to_words, oracle_mask_from_snapped, oracle_snapped,
                               words_to_i64)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def tk():
    from paper_2603_11404_amd import tk as _tk
    return _tk


def gpu_raster_from_snapped(sn_batch, meshes, cam):
    T = tk()
    B = sn_batch.shape[0]
    dm = [T.DeviceMesh(m, DEV) for m in meshes]
    sn = torch.as_tensor(np.ascontiguousarray(sn_batch, np.int32), device=DEV)
    masks = torch.full((B, *T.words_shape(cam)), -1, dtype=torch.int64, device=DEV)  # garbage-filled
    T.raster_from_snapped(sn, B, dm, cam, masks)
    torch.cuda.synchronize()
    return i64_to_words(masks.cpu().numpy())


def _check_batch(thetas, chain, mesh, cam):
    sns, fls = zip(*[oracle_snapped(th, chain, mesh, cam) for th in thetas])
    got = gpu_raster_from_snapped(np.stack(sns), [mesh], cam)
    for k in range(len(thetas)):
        ref = oracle_mask_from_snapped(sns[k], fls[k], mesh, cam)
        if not np.array_equal(got[k], ref):
            img_g = scenes.words_to_image(got[k], cam.width, cam.height)
            img_r = scenes.words_to_image(ref, cam.width, cam.height)
            pytest.fail(f"candidate {k}: {int((img_g ^ img_r).sum())} pixels differ "
                        f"(gpu {int(img_g.sum())}, oracle {int(img_r.sum())})")


@pytest.mark.parametrize("name", ["small", "track640"])
def test_raster_from_snapped_bit_exact_workloads(name):
    wl = scenes.workload(name)
    rng = np.random.default_rng(100 + wl["index"])
    th = candidates(rng, wl["cam"], 24, spread=3.0)
    _check_batch(th, scenes.chain(), wl["mesh"], wl["cam"])


@pytest.mark.parametrize("W,H,f", [(13, 11, 12.0), (100, 75, 90.0), (333, 197, 300.0), (1280, 720, 1600.0)])
def test_raster_from_snapped_ragged_and_large_images(W, H, f):
    cam = scenes.camera(W, H, f)
    mesh = scenes.instrument_mesh(32, 28, 3, 1)
    rng = np.random.default_rng(W * 7 + H)
    th = candidates(rng, cam, 6, spread=4.0)
    _check_batch(th, scenes.chain(), mesh, cam)


def test_raster_synthetic_triangles_edge_cases():
    """Random triangles of every size (sub-pixel to guard-band), ties on pixel
    centres, degenerate and flagged vertices, off-screen geometry."""
    cam = scenes.camera(200, 150, 250.0)
    rng = np.random.default_rng(7)
    nv, nt, B = 600, 400, 4
    sns = []
    for b in range(B):
        v = np.empty((nv, 2))
        scale = rng.choice([0.5, 3, 20, 150, 5000, 30000], size=nv)
        centre = rng.uniform(-30, 230, size=(nv, 2))
        v = centre + rng.normal(size=(nv, 2)) * scale[:, None]
        k = rng.random(nv)
        v[k < 0.25] = np.floor(v[k < 0.25]) + 0.5           # on pixel centres
        v[(k > 0.25) & (k < 0.35)] = np.floor(v[(k > 0.25) & (k < 0.35)])
        v = np.clip(v, -32768, 32768)
        sn = np.rint(v * 256).astype(np.int32)
        flag = rng.random(nv) < 0.03
        sn[flag, 0] = INT32_MIN
        sn[flag, 1] = 0
        sns.append(sn)
    tris = rng.integers(0, nv, size=(nt, 3)).astype(np.int32)
    tris[:10, 1] = tris[:10, 0]                                 # degenerate
    mesh = scenes.Mesh(np.zeros((nv, 3), np.float32), tris, np.zeros(nv, np.uint8), {})
    got = gpu_raster_from_snapped(np.stack(sns), [mesh], cam)
    for b in range(B):
        fl = (sns[b][:, 0] == INT32_MIN).astype(np.uint8)
        ref = oracle_mask_from_snapped(sns[b], fl, mesh, cam)
        np.testing.assert_array_equal(got[b], ref, err_msg=f"batch {b}")


def test_raster_two_meshes_union_and_empty():
    cam = scenes.camera(320, 240, 400.0)
    m1 = scenes.instrument_mesh(32, 28, 3, 1)
    m2 = scenes.instrument_mesh(32, 10, 2, 1, jaw_scale=1.3, box_scale=1.2)
    ch = scenes.chain()
    rng = np.random.default_rng(21)
    th1 = candidates(rng, cam, 3)
    th2 = candidates(rng, cam, 3)
    sn = []
    refs = []
    for k in range(3):
        s1, f1 = oracle_snapped(th1[k], ch, m1, cam)
        s2, f2 = oracle_snapped(th2[k], ch, m2, cam)
        sn.append(np.concatenate([s1, s2]))
        ref = oracle_mask_from_snapped(s1, f1, m1, cam) | oracle_mask_from_snapped(s2, f2, m2, cam)
        refs.append(ref)
    got = gpu_raster_from_snapped(np.stack(sn), [m1, m2], cam)
    for k in range(3):
        np.testing.assert_array_equal(got[k], refs[k])
    # a mesh with no triangles renders nothing
    empty = scenes.Mesh(m1.vertices, np.zeros((0, 3), np.int32), m1.vertex_link, {})
    got = gpu_raster_from_snapped(np.stack(sn)[:, :m1.n_vertices], [empty], cam)
    assert not got.any()
    # beside a mesh that has triangles, either arm may be the empty one
    # (triangle chunks are numbered over both meshes)
    s1 = np.stack(sn)[:, :m1.n_vertices]
    s2 = np.stack(sn)[:, m1.n_vertices:]
    only2 = [oracle_mask_from_snapped(*oracle_snapped(th2[k], ch, m2, cam), m2, cam) for k in range(3)]
    only1 = [oracle_mask_from_snapped(*oracle_snapped(th1[k], ch, m1, cam), m1, cam) for k in range(3)]
    empty2 = scenes.Mesh(m2.vertices, np.zeros((0, 3), np.int32), m2.vertex_link, {})
    got = gpu_raster_from_snapped(np.concatenate([s1, s2], axis=1), [empty, m2], cam)
    for k in range(3):
        np.testing.assert_array_equal(got[k], only2[k])
    got = gpu_raster_from_snapped(np.concatenate([s1, s2], axis=1), [m1, empty2], cam)
    for k in range(3):
        np.testing.assert_array_equal(got[k], only1[k])


def test_mask_counts_bit_exact():
    T = tk()
    rng = np.random.default_rng(3)
    for W, H in [(640, 480), (13, 9), (961, 541)]:
        cam = scenes.camera(W, H)
        B = 5
        imgs = rng.random((B, H, W)) < rng.uniform(0.01, 0.6, size=(B, 1, 1))
        words = scenes.image_to_words(imgs)
        pad = ~scenes.image_to_words(np.ones((H, W), bool))        # bits of pixels outside the image
        words |= pad[None] & rng.integers(0, 2 ** 63, size=words.shape, dtype=np.uint64)   # must be ignored
        tgt_img = rng.random((H, W)) < 0.2
        tgt = scenes.image_to_words(tgt_img)
        masks = torch.as_tensor(words_to_i64(words), device=DEV)
        target = torch.as_tensor(words_to_i64(tgt), device=DEV)
        counts = torch.empty(B, 2, dtype=torch.int32, device=DEV)
        pc = torch.empty(B, dtype=torch.int32, device=DEV)
        T.mask_loss(masks, B, target, cam, counts)
        T.mask_popcount(masks, B, cam, pc)
        torch.cuda.synchronize()
        c = counts.cpu().numpy()
        for b in range(B):
            assert c[b, 0] == imgs[b].sum() and c[b, 1] == (imgs[b] & tgt_img).sum()
            assert pc.cpu().numpy()[b] == imgs[b].sum()


def test_fused_equals_plain_and_oracle_counts():
    """The GPU forms of the path agree bit for bit: tk_eval_fused counts equal
    tk_raster_silhouette + tk_mask_loss counts, and tk_snap_vertices +
    tk_raster_from_snapped reproduces the tk_raster_silhouette masks (their
    agreement with the oracle given the same snapped vertices is tested above)."""
    T = tk()
    wl = scenes.workload("track640")
    mesh, cam = wl["mesh"], wl["cam"]
    ch = scenes.chain()
    rng = np.random.default_rng(55)
    B = 64
    X = torch.as_tensor(candidates(rng, cam, B, spread=2.0), device=DEV)
    xf = torch.empty(B, 1, 4, 12, dtype=torch.float32, device=DEV)
    T.fk_transform(X, B, 1, [ch], xf)
    dm = T.DeviceMesh(mesh, DEV)
    truth = scenes.true_pose(np.random.default_rng(56), cam)
    tgt = oracle.render(truth, [ch], [mesh], cam)
    target = torch.as_tensor(words_to_i64(tgt), device=DEV)
    masks = torch.empty(B, *T.words_shape(cam), dtype=torch.int64, device=DEV)
    T.raster_silhouette(xf, B, [dm], cam, masks)
    c_plain = torch.empty(B, 2, dtype=torch.int32, device=DEV)
    T.mask_loss(masks, B, target, cam, c_plain)
    c_fused = torch.empty(B, 2, dtype=torch.int32, device=DEV)
    T.eval_fused(xf, B, [dm], cam, target, c_fused)
    # the workspace forms (vertices snapped once per candidate) give the same bits
    ws = T.raster_workspace(B, [dm], DEV)
    masks_ws = torch.empty_like(masks)
    T.raster_silhouette(xf, B, [dm], cam, masks_ws, ws)
    c_fused_ws = torch.empty(B, 2, dtype=torch.int32, device=DEV)
    T.eval_fused(xf, B, [dm], cam, target, c_fused_ws, ws)
    # plain per-vertex snap + raster_from_snapped gives the same masks again
    sn = torch.empty(B, mesh.n_vertices, 2, dtype=torch.int32, device=DEV)
    T.snap_vertices(xf, B, [dm], cam, sn)
    masks2 = torch.empty_like(masks)
    T.raster_from_snapped(sn, B, [dm], cam, masks2)
    torch.cuda.synchronize()
    assert torch.equal(c_plain, c_fused)
    assert torch.equal(c_plain, c_fused_ws)
    assert torch.equal(masks, masks2)
    assert torch.equal(masks, masks_ws)
    assert int(c_plain[:, 0].max()) > 0


def test_full_path_masks_differ_only_at_edges():
    """FP32 GPU transform vs FP64 oracle: every pixel where the GPU mask and the
    oracle mask (each from its own transform) differ lies within 0.05 px of an
    edge of an oracle triangle."""
    T = tk()
    wl = scenes.workload("track640")
    mesh, cam = wl["mesh"], wl["cam"]
    ch = scenes.chain()
    rng = np.random.default_rng(77)
    B = 8
    th = candidates(rng, cam, B, spread=2.0)
    X = torch.as_tensor(th, device=DEV)
    xf = torch.empty(B, 1, 4, 12, dtype=torch.float32, device=DEV)
    T.fk_transform(X, B, 1, [ch], xf)
    dm = T.DeviceMesh(mesh, DEV)
    masks = torch.empty(B, *T.words_shape(cam), dtype=torch.int64, device=DEV)
    T.raster_silhouette(xf, B, [dm], cam, masks)
    torch.cuda.synchronize()
    got = i64_to_words(masks.cpu().numpy())
    total_diff = 0
    for k in range(B):
        sn, fl = oracle_snapped(th[k], ch, mesh, cam)
        ref = oracle_mask_from_snapped(sn, fl, mesh, cam)
        diff = scenes.words_to_image(got[k] ^ ref, cam.width, cam.height)
        ys, xs = np.nonzero(diff)
        total_diff += len(ys)
        if not len(ys):
            continue
        M = oracle.fk(th[k].astype(np.float64), ch)
        uv, _, flags = oracle.project_snap(M, mesh, cam)
        tri = mesh.triangles[~flags[mesh.triangles].any(1)]
        P = uv[tri]                                          # [T,3,2] float64 pixel coordinates
        for y, x in zip(ys, xs):
            c = np.array([x + 0.5, y + 0.5])
            best = np.inf
            for e in range(3):
                a, b = P[:, e], P[:, (e + 1) % 3]
                d = b - a
                L2 = (d ** 2).sum(1)
                t = np.clip(((c - a) * d).sum(1) / np.where(L2 > 0, L2, 1), 0, 1)
                dist = np.linalg.norm(a + t[:, None] * d - c, axis=1)
                best = min(best, dist.min())
            assert best < 0.05, f"candidate {k} pixel ({x},{y}) is {best:.3f} px from every edge"
    assert total_diff < 0.001 * B * cam.width * cam.height


def test_invalid_arguments_raise_without_launch():
    T = tk()
    cam = scenes.camera(320, 240)
    mesh = T.DeviceMesh(scenes.instrument_mesh(8, 2, 1, 1), DEV)
    xf = torch.zeros(2, 1, 4, 12, device=DEV)
    masks = torch.empty(2, *T.words_shape(cam), dtype=torch.int64, device=DEV)
    with pytest.raises(T.TkError) as e:
        T.raster_silhouette(xf, -1, [mesh], cam, masks)
    assert e.value.status == 1
    bad = scenes.camera(5000, 10)
    with pytest.raises(T.TkError):
        T.raster_silhouette(xf, 2, [mesh], bad, masks)
    too_big = scenes.camera(2000, 1500)
    with pytest.raises(T.TkError) as e:
        T.raster_silhouette(xf, 2, [mesh], too_big, torch.empty(2, 188, 250, dtype=torch.int64, device=DEV))
    assert e.value.status == 2
    T.raster_silhouette(xf, 0, [mesh], cam, masks)        # empty batch is a no-op
    small_ws = torch.empty(8, dtype=torch.uint8, device=DEV)
    with pytest.raises(T.TkError) as e:
        T.raster_silhouette(xf, 2, [mesh], cam, masks, small_ws)
    assert e.value.status == 3


@pytest.mark.parametrize("name", ["small", "track640"])
def test_claim_order_renders_the_same_masks(name):
    """The same snapped vertices rasterised from the mesh as given and from its
    tk_mesh_chunk_order copy: identical masks, equal to the oracle's (which
    reads the triangles as given)."""
    T = tk()
    wl = scenes.workload(name)
    mesh, cam = wl["mesh"], wl["cam"]
    rng = np.random.default_rng(300 + wl["index"])
    th = candidates(rng, cam, 12, spread=3.0)
    sns, fls = zip(*[oracle_snapped(t, scenes.chain(), mesh, cam) for t in th])
    sn = torch.as_tensor(np.ascontiguousarray(np.stack(sns), np.int32), device=DEV)
    got = []
    for order in (False, True):
        dm = T.DeviceMesh(mesh, DEV, chunk_order=order)
        masks = torch.full((len(th), *T.words_shape(cam)), -1, dtype=torch.int64, device=DEV)
        T.raster_from_snapped(sn, len(th), [dm], cam, masks)
        torch.cuda.synchronize()
        got.append(i64_to_words(masks.cpu().numpy()))
    np.testing.assert_array_equal(got[0], got[1])
    for k in range(len(th)):
        np.testing.assert_array_equal(got[1][k], oracle_mask_from_snapped(sns[k], fls[k], mesh, cam))
