"""CPU oracle for the batched silhouette-fitness path (arXiv 2603.11404).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the bench's
CPU-baseline leg are the only callers.  The product path (the HIP library and
its binding) never imports this package, and this package never imports the
product path.

* ``tko.c`` -- FP64 forward kinematics, projection and Q8 snapping, int64
  edge-function rasterisation with the top-left rule, counts and losses
  (paper Sec. III-A.2 and III-A.3).
* ``cmaes.py`` -- FP64 CMA-ES with Philox4x32-10 + Box-Muller sampling
  (paper Sec. III-A.1, completed with Hansen's tutorial where the paper is
  silent).
* ``tko_soft.c`` -- FP64 soft silhouette (sigmoid of the signed edge
  distance, probabilistic OR over faces), its squared-error loss and the
  analytic gradient through projection, forward kinematics and the cosine
  joint map, plus the forward-kinematics Jacobian.
* ``brute.py`` -- exact rational point-in-triangle checker for tiny images.
* ``kalman.py`` -- constant-velocity Kalman filter of the per-frame estimates
  in the general 2n-state matrix form (paper Sec. III-A.4).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "tko.c")
_SRCS = [_SRC, os.path.join(_HERE, "tko_soft.c")]

BUILD_CMD = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", "-o", _SO, *_SRCS, "-lm"]


def build() -> str:
    """Compile liboracle.so with gcc (no fast-math, no FP contraction)."""
    subprocess.check_call(BUILD_CMD, cwd=_HERE)
    return _SO


class _Camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_double)]


class _Chain(ctypes.Structure):
    _fields_ = [("d_pitch_yaw", ctypes.c_double), ("q_lb", ctypes.c_double * 3),
                ("q_ub", ctypes.c_double * 3), ("keypoints", (ctypes.c_double * 4) * 4)]


class _Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_triangles", ctypes.c_int32),
                ("vertices", ctypes.c_void_p), ("triangles", ctypes.c_void_p),
                ("vertex_link", ctypes.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < max(
                os.path.getmtime(f) for f in _SRCS + [os.path.join(_HERE, "tko.h")]):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        L.tko_decode.restype = d
        L.tko_decode.argtypes = [d, d, d]
        L.tko_encode.restype = d
        L.tko_encode.argtypes = [d, d, d]
        L.tko_pose.argtypes = [d, d, d, d, d, d, P]
        L.tko_chain_links.argtypes = [P, P, P]
        L.tko_fk.argtypes = [P, P, P]
        L.tko_project_snap.argtypes = [P, P, P, i32, P, P, P, P]
        L.tko_keypoints.argtypes = [P, P, P, P]
        L.tko_raster.restype = i64
        L.tko_raster.argtypes = [P, P, i32, P, i32, i32, i32, P, P]
        L.tko_counts.argtypes = [P, P, i32, i32, P]
        L.tko_mask_loss.restype = d
        L.tko_mask_loss.argtypes = [i64, i64, i64, i32, d]
        L.tko_kp_loss.restype = d
        L.tko_kp_loss.argtypes = [P, P, d]
        L.tko_kp_loss_tips.restype = d
        L.tko_kp_loss_tips.argtypes = [P, P, d]
        L.tko_eval_batch.argtypes = [P, i32, i32, P, P, P, P, P, P, i32]
        L.tko_max_threads.restype = i32
        L.tko_fk_jacobian.argtypes = [P, P, P]
        L.tko_soft.restype = d
        L.tko_soft.argtypes = [P, i32, P, P, P, d, P, P, P]
        L.tko_soft_banded.restype = d
        L.tko_soft_banded.argtypes = [P, i32, P, P, P, d, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cam(cam) -> _Camera:
    return _Camera(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.z_near)


def _chain(ch) -> _Chain:
    c = _Chain()
    c.d_pitch_yaw = float(ch.d_pitch_yaw)
    for j in range(3):
        c.q_lb[j] = float(ch.q_lb[j])
        c.q_ub[j] = float(ch.q_ub[j])
    for j in range(4):
        for k in range(4):
            c.keypoints[j][k] = float(ch.keypoints[j][k])
    return c


# ---------------------------------------------------------------- geometry

def decode(qhat, lb, ub) -> float:
    return lib().tko_decode(float(qhat), float(lb), float(ub))


def encode(q, lb, ub) -> float:
    return lib().tko_encode(float(q), float(lb), float(ub))


def pose(alpha, beta, gamma, x, y, z) -> np.ndarray:
    T = np.zeros(12)
    lib().tko_pose(alpha, beta, gamma, x, y, z, _p(T))
    return T.reshape(3, 4)


def chain_links(q, ch) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    T = np.zeros((4, 12))
    c = _chain(ch)
    lib().tko_chain_links(_p(q), ctypes.byref(c), _p(T))
    return T.reshape(4, 3, 4)


def fk(theta, ch) -> np.ndarray:
    """theta[9] -> M[4,3,4] (FP64)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    M = np.zeros((4, 12))
    c = _chain(ch)
    lib().tko_fk(_p(th), ctypes.byref(c), _p(M))
    return M.reshape(4, 3, 4)


def project_snap(M, mesh, cam):
    """-> uv [V,2] float64, snapped [V,2] int32, flags [V] uint8."""
    M = np.ascontiguousarray(M, dtype=np.float64).reshape(4, 12)
    V = mesh.n_vertices
    uv = np.zeros((V, 2))
    sn = np.zeros((V, 2), dtype=np.int32)
    fl = np.zeros(V, dtype=np.uint8)
    c = _cam(cam)
    verts = np.ascontiguousarray(mesh.vertices, dtype=np.float32)
    vl = np.ascontiguousarray(mesh.vertex_link, dtype=np.uint8)
    lib().tko_project_snap(_p(M), _p(verts), _p(vl), V, ctypes.byref(c), _p(uv), _p(sn), _p(fl))
    return uv, sn, fl


def keypoints(M, ch, cam) -> np.ndarray:
    M = np.ascontiguousarray(M, dtype=np.float64).reshape(4, 12)
    kp = np.zeros((4, 2))
    c = _chain(ch)
    cm = _cam(cam)
    lib().tko_keypoints(_p(M), ctypes.byref(c), ctypes.byref(cm), _p(kp))
    return kp


def raster(snapped, flags, triangles, width, height, with_counts=False, mask=None):
    """Rasterise one mesh -> word mask [ceil(H/8), ceil(W/8)] (ORed into `mask` if given)."""
    sn = np.ascontiguousarray(snapped, dtype=np.int32)
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    tr = np.ascontiguousarray(triangles, dtype=np.int32)
    by, bx = (height + 7) // 8, (width + 7) // 8
    out = np.zeros((by, bx), dtype=np.uint64) if mask is None else mask
    cnt = np.zeros((height, width), dtype=np.int32) if with_counts else None
    lib().tko_raster(_p(sn), _p(fl), int(sn.shape[0]), _p(tr), int(tr.shape[0]), int(width), int(height),
                     _p(out), _p(cnt) if cnt is not None else None)
    return (out, cnt) if with_counts else out


def counts(S, Mref, width, height):
    S = np.ascontiguousarray(S, dtype=np.uint64)
    Mref = np.ascontiguousarray(Mref, dtype=np.uint64)
    out = np.zeros(3, dtype=np.int64)
    lib().tko_counts(_p(S), _p(Mref), int(width), int(height), _p(out))
    return tuple(int(v) for v in out)


def mask_loss(a, i, m, kind=0, lambda_app=1.0) -> float:
    return lib().tko_mask_loss(int(a), int(i), int(m), int(kind), float(lambda_app))


def kp_loss(kp, ref, tau=0.0) -> float:
    kp = np.ascontiguousarray(kp, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    return lib().tko_kp_loss(_p(kp), _p(ref), float(tau))


def kp_loss_tips(kp, ref, tau=0.0) -> float:
    """Keypoint loss of Eq. (8) on the two tool tips (keypoints 2, 3)."""
    kp = np.ascontiguousarray(kp, dtype=np.float64)
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    return lib().tko_kp_loss_tips(_p(kp), _p(ref), float(tau))


def render(theta_arms, chains, meshes, cam) -> np.ndarray:
    """Silhouette (word mask) of one candidate: OR over the arms' meshes."""
    theta_arms = np.asarray(theta_arms, dtype=np.float64).reshape(-1, 9)
    mask = np.zeros(((cam.height + 7) // 8, (cam.width + 7) // 8), dtype=np.uint64)
    for th, ch, me in zip(theta_arms, chains, meshes):
        M = fk(th, ch)
        _, sn, fl = project_snap(M, me, cam)
        raster(sn, fl, me.triangles, cam.width, cam.height, mask=mask)
    return mask


def eval_batch(theta, chains, meshes, cam, target, n_threads=0, want_masks=False):
    """theta [B, n_arms*9] -> counts [B,2] (|S|, |S and M|) (and masks)."""
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    B = theta.shape[0]
    n_arms = len(meshes)
    ch = (_Chain * n_arms)(*[_chain(c) for c in chains])
    keep = [(np.ascontiguousarray(m.vertices, dtype=np.float32),
             np.ascontiguousarray(m.triangles, dtype=np.int32),
             np.ascontiguousarray(m.vertex_link, dtype=np.uint8)) for m in meshes]
    me = (_Mesh * n_arms)(*[_Mesh(m.n_vertices, m.n_triangles, _p(v), _p(t), _p(l))
                            for m, (v, t, l) in zip(meshes, keep)])
    cm = _cam(cam)
    tgt = np.ascontiguousarray(target, dtype=np.uint64)
    cnt = np.zeros((B, 2), dtype=np.int64)
    words = ((cam.height + 7) // 8) * ((cam.width + 7) // 8)
    masks = np.zeros((B, (cam.height + 7) // 8, (cam.width + 7) // 8), dtype=np.uint64) if want_masks else None
    lib().tko_eval_batch(_p(theta), B, n_arms, ch, me, ctypes.byref(cm), _p(tgt), _p(cnt),
                         _p(masks) if masks is not None else None, int(n_threads))
    del words
    return (cnt, masks) if want_masks else cnt


def fk_jacobian(theta, chain) -> np.ndarray:
    """d M_l / d theta_k as [9, 4, 12] (FP64)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.zeros((9, 4, 12))
    c = _chain(chain)
    lib().tko_fk_jacobian(_p(th), ctypes.byref(c), _p(out))
    return out


def soft(theta_arms, chains, meshes, cam, sigma, target=None, want_S=False, want_grad=False, banded=False):
    """Soft silhouette loss L = sum_p (S - M)^2 of the arms at theta [n_arms*9]
    (FP64); returns (L, S [H, W] or None, dL/dtheta [n_arms*9] or None).
    banded=True evaluates the same definitions face-major over each face's
    10-sigma box (tko_soft_banded), for large meshes."""
    theta = np.ascontiguousarray(theta_arms, dtype=np.float64).reshape(-1)
    n_arms = len(meshes)
    ch = (_Chain * n_arms)(*[_chain(c) for c in chains])
    keep = [(np.ascontiguousarray(m.vertices, dtype=np.float32),
             np.ascontiguousarray(m.triangles, dtype=np.int32),
             np.ascontiguousarray(m.vertex_link, dtype=np.uint8)) for m in meshes]
    me = (_Mesh * n_arms)(*[_Mesh(m.n_vertices, m.n_triangles, _p(v), _p(t), _p(l))
                            for m, (v, t, l) in zip(meshes, keep)])
    cm = _cam(cam)
    tgt = None if target is None else np.ascontiguousarray(target, dtype=np.uint64)
    S = np.zeros((cam.height, cam.width)) if want_S else None
    g = np.zeros(9 * n_arms) if want_grad else None
    fn = lib().tko_soft_banded if banded else lib().tko_soft
    L = fn(_p(theta), n_arms, ch, me, ctypes.byref(cm), float(sigma),
                       _p(tgt) if tgt is not None else None, _p(S) if S is not None else None,
                       _p(g) if g is not None else None)
    return float(L), S, g


def max_threads() -> int:
    return int(lib().tko_max_threads())
