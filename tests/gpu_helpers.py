"""Shared helpers of the GPU parity tests (inputs come from scenes/oracle only)."""
import numpy as np

import oracle
import scenes

INT32_MIN = np.iinfo(np.int32).min


def words_to_i64(words):
    return np.ascontiguousarray(words, dtype=np.uint64).view(np.int64)


def i64_to_words(arr):
    return np.ascontiguousarray(arr, dtype=np.int64).view(np.uint64)


def oracle_snapped(theta, chain, mesh, cam):
    """FP64 oracle projection of one candidate -> (snapped with INT32_MIN flags, flags)."""
    M = oracle.fk(np.asarray(theta, np.float64), chain)
    _, sn, fl = oracle.project_snap(M, mesh, cam)
    sn = sn.copy()
    sn[fl.astype(bool), 0] = INT32_MIN
    sn[fl.astype(bool), 1] = 0
    return sn, fl


def oracle_mask_from_snapped(sn, fl, mesh, cam):
    s = np.where(fl[:, None].astype(bool), 0, sn).astype(np.int32)
    return oracle.raster(s, fl, mesh.triangles, cam.width, cam.height)


def candidates(rng, cam, n, spread=1.0):
    """Candidates around seeded true poses: theta = truth + spread * scale * N(0, I), as float32."""
    base = scenes.true_pose(rng, cam)
    th = base[None, :] + spread * scenes.DEFAULT_SCALE[None, :] * rng.normal(size=(n, 9))
    return th.astype(np.float32)
