"""Thin ctypes binding of libtk (include/tk.h): argument marshalling only.

Every step of the fitness path runs in the HIP kernels of libtk.so; torch is
used for device memory and for the current HIP stream.  The library must be
built (``python -m paper_2603_11404_amd.build``); on a machine with a GPU a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # imported before libtk so that both share torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtk.so")

TK_OK = 0
TK_ERR_INVALID_ARGUMENT, TK_ERR_UNSUPPORTED, TK_ERR_WORKSPACE_TOO_SMALL, TK_ERR_DEVICE = 1, 2, 3, 4
STATUS_NAMES = {0: "TK_OK", 1: "TK_ERR_INVALID_ARGUMENT", 2: "TK_ERR_UNSUPPORTED",
                3: "TK_ERR_WORKSPACE_TOO_SMALL", 4: "TK_ERR_DEVICE"}

LOSS_IOU, LOSS_RENDER = 0, 1
KP_TWO_TIPS = 16            # flag bit of the loss kind: the two-tip keypoint term of Eq. (8)


class TkError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("z_near", ctypes.c_float)]


class Mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_triangles", ctypes.c_int32),
                ("vertices", ctypes.c_void_p), ("triangles", ctypes.c_void_p), ("vertex_link", ctypes.c_void_p),
                ("closed", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Chain(ctypes.Structure):
    _fields_ = [("d_pitch_yaw", ctypes.c_double), ("q_lb", ctypes.c_double * 3), ("q_ub", ctypes.c_double * 3),
                ("keypoints", (ctypes.c_double * 4) * 4)]


class Problem(ctypes.Structure):
    """tk_problem: one independent problem of a batched launch."""
    _fields_ = [("d_state", ctypes.c_void_p), ("n", ctypes.c_int32), ("lambda_", ctypes.c_int32),
                ("n_arms", ctypes.c_int32), ("meshes", Mesh * 2), ("chains", Chain * 2), ("cam", Camera),
                ("d_target", ctypes.c_void_p), ("d_target_count", ctypes.c_void_p), ("d_X", ctypes.c_void_p),
                ("d_link_xf", ctypes.c_void_p), ("d_kp", ctypes.c_void_p), ("d_counts", ctypes.c_void_p),
                ("d_ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t), ("kind", ctypes.c_int32),
                ("lambda_app", ctypes.c_double), ("d_kp_ref", ctypes.c_void_p), ("lambda_kp", ctypes.c_double),
                ("tau", ctypes.c_double), ("d_loss", ctypes.c_void_p), ("threads", ctypes.c_int32)]


class CmaesParams(ctypes.Structure):
    _fields_ = [("c_m_scale", ctypes.c_double), ("c_mu_scale", ctypes.c_double), ("c1_scale", ctypes.c_double),
                ("n_blocks", ctypes.c_int32)]


_LAYOUT_FIELDS = ["total_bytes", "gen", "seed", "flags", "sigma", "c_sigma", "d_sigma", "c_c", "c1", "c_mu", "c_m",
                  "mu_eff", "chi_n", "h_sigma", "weights", "mean", "p_sigma", "p_c", "offset", "scale", "D", "C",
                  "B", "Z", "Y", "order", "z_gen", "L"]


class CmaesLayout(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in _LAYOUT_FIELDS]


EXPORTS = [
    "tk_status_string", "tk_last_error", "tk_version",
    "tk_cmaes_state_bytes", "tk_cmaes_layout_get", "tk_cmaes_init", "tk_cmaes_init_at", "tk_cmaes_set_mean",
    "tk_cmaes_sample",
    "tk_cmaes_update", "tk_fk_transform", "tk_snap_vertices", "tk_raster_silhouette", "tk_raster_from_snapped",
    "tk_mask_loss", "tk_mask_popcount", "tk_eval_fused", "tk_compose_loss", "tk_raster_stats",
    "tk_raster_workspace_bytes", "tk_cmaes_tell_ask", "tk_cmaes_tell", "tk_cmaes_ask_eval",
    "tk_cmaes_ask_eval_noalloc",
    "tk_batch_table_bytes", "tk_batch_describe", "tk_batch_ask_eval", "tk_batch_tell",
    "tk_kf_state_bytes", "tk_kf_init", "tk_kf_step", "tk_cmaes_estimate",
    "tk_soft_workspace_bytes", "tk_soft_forward", "tk_soft_backward", "tk_cmaes_mean_candidate", "tk_adam_reset",
    "tk_cmaes_adam", "tk_cmaes_adam_transform", "tk_mesh_chunk_order", "tk_mesh_closed", "tk_mesh_plane_order", "tk_bench_copy",
    "tk_bench_lds", "tk_batch_ask_eval_persistent",
]

_lib = None


def lib():
    """Load libtk.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2603_11404_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, f64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
        L.tk_status_string.restype = ctypes.c_char_p
        L.tk_status_string.argtypes = [ctypes.c_int]
        L.tk_last_error.restype = ctypes.c_char_p
        L.tk_last_error.argtypes = []
        L.tk_version.restype = i32
        L.tk_cmaes_state_bytes.restype = ctypes.c_size_t
        L.tk_cmaes_state_bytes.argtypes = [i32, i32]
        L.tk_cmaes_layout_get.argtypes = [i32, i32, P]
        L.tk_cmaes_init.argtypes = [P, i32, i32, P, f64, P, P, P, u64, P]
        L.tk_cmaes_init_at.argtypes = [P, i32, i32, P, P, i32, P, f64, P, P, u64, P]
        L.tk_cmaes_set_mean.argtypes = [P, i32, i32, P, P]
        L.tk_cmaes_sample.argtypes = [P, i32, i32, P, P]
        L.tk_cmaes_update.argtypes = [P, i32, i32, P, P]
        L.tk_fk_transform.argtypes = [P, i32, i32, P, P, P, P, P]
        L.tk_snap_vertices.argtypes = [P, i32, P, i32, P, P, P]
        L.tk_raster_workspace_bytes.restype = ctypes.c_size_t
        L.tk_raster_workspace_bytes.argtypes = [i32, P, i32]
        L.tk_raster_silhouette.argtypes = [P, i32, P, i32, P, P, P, ctypes.c_size_t, P]
        L.tk_raster_from_snapped.argtypes = [P, i32, P, i32, P, P, P]
        L.tk_mask_loss.argtypes = [P, i32, P, P, P, P]
        L.tk_mask_popcount.argtypes = [P, i32, P, P, P]
        L.tk_eval_fused.argtypes = [P, i32, P, i32, P, P, P, P, ctypes.c_size_t, P]
        L.tk_compose_loss.argtypes = [P, i32, P, i32, f64, P, P, i32, f64, f64, P, P]
        L.tk_raster_stats.argtypes = [P, i32, P, i32, P, P, P]
        L.tk_cmaes_tell_ask.argtypes = [P, i32, i32, P, P, i32, f64, P, P, f64, f64, P, P, i32, P, P, P, P, P]
        L.tk_cmaes_tell.argtypes = [P, i32, i32, P, P, i32, f64, P, P, i32, f64, f64, P, P]
        L.tk_cmaes_ask_eval.argtypes = [P, i32, i32, P, i32, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.tk_cmaes_ask_eval_noalloc.argtypes = [P, i32, i32, P, i32, P, P, P, P, P, P, P, P]
        L.tk_batch_table_bytes.restype = ctypes.c_size_t
        L.tk_batch_table_bytes.argtypes = [i32]
        L.tk_batch_describe.argtypes = [P, i32, P, ctypes.c_size_t]
        L.tk_batch_ask_eval.argtypes = [P, i32, P, P]
        L.tk_batch_ask_eval_persistent.argtypes = [P, i32, P, P]
        L.tk_batch_tell.argtypes = [P, i32, P, P]
        L.tk_kf_state_bytes.restype = ctypes.c_size_t
        L.tk_kf_state_bytes.argtypes = [i32]
        L.tk_kf_init.argtypes = [P, i32, P, P, P]
        L.tk_kf_step.argtypes = [P, i32, P, P, P, P]
        L.tk_cmaes_estimate.argtypes = [P, i32, i32, P, i32, P, P]
        f32 = ctypes.c_float
        L.tk_soft_workspace_bytes.restype = ctypes.c_size_t
        L.tk_soft_workspace_bytes.argtypes = [i32, P, i32, P]
        L.tk_soft_forward.argtypes = [P, i32, P, i32, P, f32, P, P, P, P, ctypes.c_size_t, P]
        L.tk_soft_backward.argtypes = [P, i32, P, P, i32, P, f32, P, P, P, ctypes.c_size_t, P]
        L.tk_cmaes_mean_candidate.argtypes = [P, i32, i32, P, P]
        L.tk_adam_reset.argtypes = [P, i32, P]
        L.tk_cmaes_adam.argtypes = [P, i32, i32, P, P, f64, f64, f64, f64, P]
        L.tk_cmaes_adam_transform.argtypes = [P, i32, i32, P, P, f64, f64, f64, f64, i32, P, P, P, P]
        L.tk_mesh_chunk_order.argtypes = [P, i32, P, i32, P]
        L.tk_mesh_closed.argtypes = [P, i32, i32, P]
        L.tk_bench_copy.argtypes = [P, P, ctypes.c_size_t, P]
        L.tk_bench_lds.argtypes = [i32, i32, P, P]
        L.tk_mesh_plane_order.argtypes = [P, P, i32, P, i32, P]
        for name in EXPORTS:
            if name not in ("tk_status_string", "tk_last_error", "tk_version", "tk_cmaes_state_bytes",
                            "tk_raster_workspace_bytes", "tk_batch_table_bytes", "tk_kf_state_bytes",
                            "tk_soft_workspace_bytes"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != TK_OK:
        raise TkError(status, lib().tk_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("expected a device tensor")
        if not t.is_contiguous():
            raise ValueError("expected a contiguous tensor")
        return ctypes.c_void_p(t.data_ptr())
    raise TypeError(type(t))


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def camera(cam) -> Camera:
    """tk_camera from any object with fx, fy, cx, cy, width, height, z_near."""
    return Camera(cam.fx, cam.fy, cam.cx, cam.cy, int(cam.width), int(cam.height), cam.z_near)


def chain(ch) -> Chain:
    c = Chain()
    c.d_pitch_yaw = float(ch.d_pitch_yaw)
    for j in range(3):
        c.q_lb[j] = float(ch.q_lb[j])
        c.q_ub[j] = float(ch.q_ub[j])
    for j in range(4):
        for k in range(4):
            c.keypoints[j][k] = float(ch.keypoints[j][k])
    return c


def mesh_chunk_order(vertices, triangles) -> np.ndarray:
    """tk_mesh_chunk_order on host arrays: the same triangles [T, 3] int32 in
    the raster kernels' claim order (costly 64-triangle blocks first)."""
    v = np.ascontiguousarray(vertices, np.float32)
    t = np.ascontiguousarray(triangles, np.int32)
    out = np.empty_like(t)
    _check(lib().tk_mesh_chunk_order(v.ctypes.data, int(v.shape[0]), t.ctypes.data, int(t.shape[0]),
                                     out.ctypes.data))
    return out


def mesh_closed(triangles, n_vertices) -> bool:
    """tk_mesh_closed: whether the triangle list is a closed, consistently
    oriented surface (every directed edge matched by its reverse)."""
    t = np.ascontiguousarray(triangles, np.int32)
    out = ctypes.c_int32(-1)
    _check(lib().tk_mesh_closed(t.ctypes.data if t.size else None, int(t.shape[0]), int(n_vertices),
                                ctypes.byref(out)))
    return bool(out.value)


def mesh_plane_order(vertices, vertex_link, triangles) -> np.ndarray:
    """tk_mesh_plane_order on host arrays: the same triangles grouped by their
    supporting plane."""
    v = np.ascontiguousarray(vertices, np.float32)
    l = np.ascontiguousarray(vertex_link, np.uint8)
    t = np.ascontiguousarray(triangles, np.int32)
    out = np.empty_like(t)
    _check(lib().tk_mesh_plane_order(v.ctypes.data, l.ctypes.data, int(v.shape[0]), t.ctypes.data, int(t.shape[0]),
                                     out.ctypes.data))
    return out


class DeviceMesh:
    """Mesh arrays resident on the device plus the tk_mesh view of them.

    By default the triangles are stored grouped by plane (tk_mesh_plane_order)
    and then in the claim order of tk_mesh_chunk_order: the same silhouette,
    with mostly one-orientation chunks claimed costly ones first.  The soft
    silhouette's face-major passes prefer neighbouring faces in neighbouring
    lanes (plane_order=False keeps the list order inside the 64-triangle
    blocks).  closed is what tk_mesh_closed reports for the triangles."""

    def __init__(self, mesh, device="cuda", chunk_order=True, plane_order=True):
        tris = np.ascontiguousarray(mesh.triangles, np.int32)
        if plane_order and tris.shape[0]:
            tris = mesh_plane_order(mesh.vertices, mesh.vertex_link, tris)
        if chunk_order and tris.shape[0]:
            tris = mesh_chunk_order(mesh.vertices, tris)
        self.closed = mesh_closed(tris, mesh.n_vertices)
        self.vertices = torch.as_tensor(np.ascontiguousarray(mesh.vertices, np.float32), device=device)
        self.triangles = torch.as_tensor(tris, device=device)
        self.vertex_link = torch.as_tensor(np.ascontiguousarray(mesh.vertex_link, np.uint8), device=device)
        self.n_vertices = int(self.vertices.shape[0])
        self.n_triangles = int(self.triangles.shape[0])

    def struct(self) -> Mesh:
        return Mesh(self.n_vertices, self.n_triangles, self.vertices.data_ptr(),
                    self.triangles.data_ptr() if self.n_triangles else None, self.vertex_link.data_ptr(),
                    int(self.closed), 0)


def _meshes(meshes):
    arr = (Mesh * len(meshes))(*[m.struct() for m in meshes])
    return arr, len(meshes)


def words_shape(cam) -> tuple[int, int]:
    return ((int(cam.height) + 7) // 8, (int(cam.width) + 7) // 8)


# ------------------------------------------------------------------ CMA-ES

def cmaes_state_bytes(n: int, lam: int) -> int:
    return int(lib().tk_cmaes_state_bytes(n, lam))


def cmaes_layout(n: int, lam: int) -> dict:
    L = CmaesLayout()
    _check(lib().tk_cmaes_layout_get(n, lam, ctypes.byref(L)))
    return {f: int(getattr(L, f)) for f in _LAYOUT_FIELDS}


def cmaes_alloc(n: int, lam: int, device="cuda") -> torch.Tensor:
    """A device state blob (uint8 tensor, 256-byte aligned by the caching allocator)."""
    t = torch.zeros(cmaes_state_bytes(n, lam), dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def cmaes_init(state, n, lam, mean0, sigma0, offset, scale, seed, c_m_scale=1.0, c_mu_scale=1.0, c1_scale=1.0,
               n_blocks=1, stream=None):
    m = np.ascontiguousarray(mean0, np.float64)
    o = np.ascontiguousarray(offset, np.float64)
    s = np.ascontiguousarray(scale, np.float64)
    p = CmaesParams(c_m_scale, c_mu_scale, c1_scale, n_blocks)
    _check(lib().tk_cmaes_init(_ptr(state), n, lam, m.ctypes.data_as(ctypes.c_void_p), float(sigma0),
                               o.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p),
                               ctypes.byref(p), int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream)))


def cmaes_init_at(state, n, lam, est, chains, readings, sigma0, scale, seed, c_m_scale=1.0, c_mu_scale=1.0,
                  c1_scale=1.0, n_blocks=1, stream=None):
    """cmaes_init with mean0 = 0 and the offset taken on the device from est
    (device FP64 [n], filter coordinates: pose, joint angles), the joint
    angles encoded by the inverse cosine map; readings (host [n_arms, 3]
    unconstrained joint coordinates, or None) replace the joint offsets."""
    n_arms = len(chains)
    ch = (Chain * n_arms)(*[chain(c) for c in chains])
    r = None if readings is None else np.ascontiguousarray(readings, np.float64).reshape(-1)
    sc = np.ascontiguousarray(scale, np.float64)
    p = CmaesParams(c_m_scale, c_mu_scale, c1_scale, n_blocks)
    _check(lib().tk_cmaes_init_at(_ptr(state), n, lam, _ptr(est), ch, n_arms,
                                  r.ctypes.data_as(ctypes.c_void_p) if r is not None else None, float(sigma0),
                                  sc.ctypes.data_as(ctypes.c_void_p), ctypes.byref(p),
                                  int(seed) & 0xFFFFFFFFFFFFFFFF, _stream(stream)))


def cmaes_set_mean(state, n, lam, mean, stream=None):
    m = np.ascontiguousarray(mean, np.float64)
    _check(lib().tk_cmaes_set_mean(_ptr(state), n, lam, m.ctypes.data_as(ctypes.c_void_p), _stream(stream)))


def cmaes_sample(state, n, lam, X, stream=None):
    _check(lib().tk_cmaes_sample(_ptr(state), n, lam, _ptr(X), _stream(stream)))


def cmaes_update(state, n, lam, loss, stream=None):
    _check(lib().tk_cmaes_update(_ptr(state), n, lam, _ptr(loss), _stream(stream)))


def cmaes_tell_ask(state, n, lam, counts, target_count, kind, chains, cam, X, link_xf, kp=None, kp_ref=None,
                   lambda_app=1.0, lambda_kp=0.0, tau=0.0, loss=None, kp_next=None, stream=None):
    """One fused generation step: compose the losses from the counts (and
    keypoints), update the state, sample the next candidates into X and
    evaluate their forward kinematics into link_xf (and kp_next)."""
    n_arms = len(chains)
    ch = (Chain * n_arms)(*[chain(c) for c in chains])
    c = camera(cam)
    _check(lib().tk_cmaes_tell_ask(_ptr(state), n, lam, _ptr(counts), _ptr(target_count), int(kind),
                                   float(lambda_app), _ptr(kp), _ptr(kp_ref), float(lambda_kp), float(tau),
                                   _ptr(loss), ch, n_arms, ctypes.byref(c), _ptr(X), _ptr(link_xf), _ptr(kp_next),
                                   _stream(stream)))


def cmaes_tell(state, n, lam, counts, target_count, kind, n_arms=1, kp=None, kp_ref=None, lambda_app=1.0,
               lambda_kp=0.0, tau=0.0, loss=None, stream=None):
    """Compose the losses from the counts (and keypoints) and update the state, in one launch."""
    _check(lib().tk_cmaes_tell(_ptr(state), n, lam, _ptr(counts), _ptr(target_count), int(kind), float(lambda_app),
                               _ptr(kp), _ptr(kp_ref), int(n_arms), float(lambda_kp), float(tau), _ptr(loss),
                               _stream(stream)))


def cmaes_ask_eval(state, n, lam, chains, meshes, cam, target, X, link_xf, counts, kp=None, ws=None, stream=None):
    """Draw the generation's candidates, evaluate their FK and their fused raster counts, in one launch."""
    n_arms = len(chains)
    ch = (Chain * n_arms)(*[chain(c) for c in chains])
    arr, nm = _meshes(meshes)
    c = camera(cam)
    wp, wb = _ws(ws)
    _check(lib().tk_cmaes_ask_eval(_ptr(state), n, lam, ch, n_arms, arr, ctypes.byref(c), _ptr(target), _ptr(X),
                                   _ptr(link_xf), _ptr(kp), _ptr(counts), wp, wb, _stream(stream)))


NOALLOC_SCRATCH_BYTES = 32 * 1024 * 1024   # TK_NOALLOC_SCRATCH_BYTES


def bench_copy(src, dst, nbytes, stream=None):
    """tk_bench_copy: streaming copy of nbytes from src to dst (device tensors)."""
    _check(lib().tk_bench_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)))


def bench_lds(workgroups, iters, out, stream=None):
    """tk_bench_lds: LDS read/write loop; out: device int32 [workgroups], cleared by the caller."""
    _check(lib().tk_bench_lds(int(workgroups), int(iters), _ptr(out), _stream(stream)))


def cmaes_ask_eval_noalloc(state, n, lam, chains, meshes, cam, target, X, link_xf, counts, kp=None, stream=None):
    """cmaes_ask_eval with the library's static per-device scratch as its
    workspace: the call allocates nothing (lam x total vertices x 8 bytes
    must fit NOALLOC_SCRATCH_BYTES; overlapping calls on one device race)."""
    n_arms = len(chains)
    ch = (Chain * n_arms)(*[chain(c) for c in chains])
    arr, nm = _meshes(meshes)
    c = camera(cam)
    _check(lib().tk_cmaes_ask_eval_noalloc(_ptr(state), n, lam, ch, n_arms, arr, ctypes.byref(c), _ptr(target),
                                           _ptr(X), _ptr(link_xf), _ptr(kp), _ptr(counts), _stream(stream)))


KF_MAX_N = 18


class KfParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double)] + [(f, ctypes.c_double * KF_MAX_N) for f in
                                             ("p0_pos", "p0_vel", "q_pos", "q_cross", "q_vel", "r", "lo", "hi")]


def kf_params(n, dt, p0_pos, p0_vel, q_pos, q_vel, r, lo=None, hi=None, q_cross=0.0) -> KfParams:
    """tk_kf_params from per-coordinate values (scalars broadcast to n)."""
    p = KfParams()
    p.dt = float(dt)
    vals = {"p0_pos": p0_pos, "p0_vel": p0_vel, "q_pos": q_pos, "q_cross": q_cross, "q_vel": q_vel, "r": r,
            "lo": -np.inf if lo is None else lo, "hi": np.inf if hi is None else hi}
    for name, v in vals.items():
        arr = np.broadcast_to(np.asarray(v, np.float64), (n,))
        getattr(p, name)[:n] = [float(a) for a in arr]
    return p


def kf_alloc(n: int, device="cuda") -> torch.Tensor:
    nb = int(lib().tk_kf_state_bytes(n))
    if nb == 0:
        raise TkError(TK_ERR_INVALID_ARGUMENT, f"tk_kf_state_bytes: n = {n} outside 1..{KF_MAX_N}")
    return torch.zeros(nb, dtype=torch.uint8, device=device)


def kf_init(kf, n, x0, params: KfParams, stream=None):
    """Restart the temporal filter at x0 (host [n]) with zero velocity."""
    x = np.ascontiguousarray(x0, np.float64)
    _check(lib().tk_kf_init(_ptr(kf), n, x.ctypes.data_as(ctypes.c_void_p), ctypes.byref(params), _stream(stream)))


def kf_step(kf, n, z, theta=None, theta_next=None, stream=None):
    """Predict, update with z (device FP64 [n]) and clamp; filtered theta and
    the next frame's prediction go to the optional device outputs."""
    _check(lib().tk_kf_step(_ptr(kf), n, _ptr(z), _ptr(theta), _ptr(theta_next), _stream(stream)))


def cmaes_estimate(state, n, lam, chains, z, stream=None):
    """The CMA-ES mean as physical coordinates with joint angles (device FP64 [n])."""
    n_arms = len(chains)
    ch = (Chain * n_arms)(*[chain(c) for c in chains])
    _check(lib().tk_cmaes_estimate(_ptr(state), n, lam, ch, n_arms, _ptr(z), _stream(stream)))


def cmaes_view(state: torch.Tensor, n: int, lam: int) -> dict:
    """Named views (host copies) of a state blob's fields, for tests and checkpoints."""
    L = cmaes_layout(n, lam)
    raw = state.detach().cpu().numpy()

    def f64(off, count):
        return raw[off:off + 8 * count].view(np.float64).copy()
    out = {name: float(f64(L[name], 1)[0]) for name in
           ("sigma", "c_sigma", "d_sigma", "c_c", "c1", "c_mu", "c_m", "mu_eff", "chi_n", "h_sigma")}
    out["gen"] = int(raw[L["gen"]:L["gen"] + 8].view(np.int64)[0])
    out["flags"] = int(raw[L["flags"]:L["flags"] + 4].view(np.int32)[0])
    out["z_gen"] = int(raw[L["z_gen"]:L["z_gen"] + 8].view(np.int64)[0])
    out["weights"] = f64(L["weights"], lam)
    for name in ("mean", "p_sigma", "p_c", "offset", "scale", "D"):
        out[name] = f64(L[name], n)
    for name in ("C", "B", "L"):
        out[name] = f64(L[name], n * n).reshape(n, n)
    for name in ("Z", "Y"):
        out[name] = f64(L[name], lam * n).reshape(lam, n)
    out["order"] = raw[L["order"]:L["order"] + 4 * lam].view(np.int32).copy()
    return out


def cmaes_write(state: torch.Tensor, n: int, lam: int, **fields):
    """Overwrite FP64 fields of a state blob (e.g. restore a checkpoint or load
    a given C, L).  Synchronous host-to-device copies."""
    L = cmaes_layout(n, lam)
    for name, val in fields.items():
        if name in ("gen", "z_gen"):
            arr = np.array([int(val)], np.int64).view(np.uint8)
        else:
            arr = np.ascontiguousarray(val, np.float64).reshape(-1).view(np.uint8)
        state[L[name]:L[name] + arr.size].copy_(torch.from_numpy(arr.copy()).to(state.device))
    if "Z" in fields and "z_gen" not in fields:
        # the written z are not the draws of a known generation
        arr = np.array([-1], np.int64).view(np.uint8)
        state[L["z_gen"]:L["z_gen"] + 8].copy_(torch.from_numpy(arr.copy()).to(state.device))


# ------------------------------------------------------------------ fitness path

def fk_transform(X, batch, n_arms, chains, link_xf, kp=None, cam=None, stream=None):
    ch = (Chain * n_arms)(*[chain(c) for c in chains])
    c = camera(cam) if cam is not None else None
    _check(lib().tk_fk_transform(_ptr(X), batch, n_arms, ch, _ptr(link_xf), _ptr(kp),
                                 ctypes.byref(c) if c is not None else None, _stream(stream)))


def snap_vertices(link_xf, batch, meshes, cam, snapped, stream=None):
    arr, nm = _meshes(meshes)
    c = camera(cam)
    _check(lib().tk_snap_vertices(_ptr(link_xf), batch, arr, nm, ctypes.byref(c), _ptr(snapped), _stream(stream)))


def raster_workspace_bytes(batch, meshes) -> int:
    arr, nm = _meshes(meshes)
    return int(lib().tk_raster_workspace_bytes(batch, arr, nm))


def raster_workspace(batch, meshes, device="cuda") -> torch.Tensor:
    """A device workspace for tk_raster_silhouette / tk_eval_fused."""
    return torch.empty(max(raster_workspace_bytes(batch, meshes), 8), dtype=torch.uint8, device=device)


def _ws(ws):
    return (None, 0) if ws is None else (_ptr(ws), ws.numel() * ws.element_size())


# ------------------------------------------------------------------ differentiable form

def soft_workspace_bytes(batch, meshes, cam) -> int:
    arr, nm = _meshes(meshes)
    c = camera(cam)
    return int(lib().tk_soft_workspace_bytes(batch, arr, nm, ctypes.byref(c)))


def soft_workspace(batch, meshes, cam, device="cuda") -> torch.Tensor:
    """A 256-byte aligned device workspace for tk_soft_forward / tk_soft_backward."""
    nb = soft_workspace_bytes(batch, meshes, cam)
    if nb == 0:
        raise TkError(TK_ERR_INVALID_ARGUMENT, "tk_soft_workspace_bytes: invalid shapes " + lib().tk_last_error().decode())
    t = torch.empty(nb, dtype=torch.uint8, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def soft_forward(link_xf, batch, meshes, cam, sigma, target, loss, ws, S=None, stream=None):
    """Soft silhouette loss [batch] FP64 (and S [batch, H, W] FP32) of the link transforms."""
    arr, nm = _meshes(meshes)
    c = camera(cam)
    wp, wb = _ws(ws)
    _check(lib().tk_soft_forward(_ptr(link_xf), batch, arr, nm, ctypes.byref(c), float(sigma), _ptr(target),
                                 _ptr(S), _ptr(loss), wp, wb, _stream(stream)))


def soft_backward(X, batch, chains, meshes, cam, sigma, grad_X, ws, grad_loss=None, stream=None):
    """dL/dtheta [batch, 9 n_arms] FP32 of the last soft_forward on ws (scaled by grad_loss [batch] FP64)."""
    arr, nm = _meshes(meshes)
    ch = (Chain * nm)(*[chain(x) for x in chains])
    c = camera(cam)
    wp, wb = _ws(ws)
    _check(lib().tk_soft_backward(_ptr(X), batch, ch, arr, nm, ctypes.byref(c), float(sigma), _ptr(grad_loss),
                                  _ptr(grad_X), wp, wb, _stream(stream)))


def cmaes_mean_candidate(state, n, lam, X, stream=None):
    _check(lib().tk_cmaes_mean_candidate(_ptr(state), n, lam, _ptr(X), _stream(stream)))


def adam_alloc(n, device="cuda") -> torch.Tensor:
    return torch.zeros(2 * n + 1, dtype=torch.float64, device=device)


def adam_reset(adam, n, stream=None):
    _check(lib().tk_adam_reset(_ptr(adam), n, _stream(stream)))


def cmaes_adam(state, n, lam, grad_theta, adam, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().tk_cmaes_adam(_ptr(state), n, lam, _ptr(grad_theta), _ptr(adam), float(lr), float(beta1),
                               float(beta2), float(eps), _stream(stream)))


def cmaes_adam_transform(state, n, lam, grad_theta, adam, chains, X, link_xf=None, lr=0.1, beta1=0.9,
                         beta2=0.999, eps=1e-8, stream=None):
    ch = (Chain * len(chains))(*[chain(c) for c in chains])
    _check(lib().tk_cmaes_adam_transform(_ptr(state), n, lam, _ptr(grad_theta), _ptr(adam), float(lr), float(beta1),
                                         float(beta2), float(eps), len(chains), ch, _ptr(X), _ptr(link_xf),
                                         _stream(stream)))


def raster_silhouette(link_xf, batch, meshes, cam, masks, ws=None, stream=None):
    arr, nm = _meshes(meshes)
    c = camera(cam)
    wp, wb = _ws(ws)
    _check(lib().tk_raster_silhouette(_ptr(link_xf), batch, arr, nm, ctypes.byref(c), _ptr(masks), wp, wb,
                                      _stream(stream)))


def raster_from_snapped(snapped, batch, meshes, cam, masks, stream=None):
    arr, nm = _meshes(meshes)
    c = camera(cam)
    _check(lib().tk_raster_from_snapped(_ptr(snapped), batch, arr, nm, ctypes.byref(c), _ptr(masks),
                                        _stream(stream)))


def mask_loss(masks, batch, target, cam, counts, stream=None):
    c = camera(cam)
    _check(lib().tk_mask_loss(_ptr(masks), batch, _ptr(target), ctypes.byref(c), _ptr(counts), _stream(stream)))


def mask_popcount(masks, batch, cam, count, stream=None):
    c = camera(cam)
    _check(lib().tk_mask_popcount(_ptr(masks), batch, ctypes.byref(c), _ptr(count), _stream(stream)))


def eval_fused(link_xf, batch, meshes, cam, target, counts, ws=None, stream=None):
    arr, nm = _meshes(meshes)
    c = camera(cam)
    wp, wb = _ws(ws)
    _check(lib().tk_eval_fused(_ptr(link_xf), batch, arr, nm, ctypes.byref(c), _ptr(target), _ptr(counts), wp, wb,
                               _stream(stream)))


def compose_loss(counts, batch, target_count, kind, loss, lambda_app=1.0, kp=None, kp_ref=None, n_arms=1,
                 lambda_kp=0.0, tau=0.0, stream=None):
    _check(lib().tk_compose_loss(_ptr(counts), batch, _ptr(target_count), int(kind), float(lambda_app), _ptr(kp),
                                 _ptr(kp_ref), int(n_arms), float(lambda_kp), float(tau), _ptr(loss),
                                 _stream(stream)))


def raster_stats(link_xf, batch, meshes, cam, stats, stream=None):
    """stats: int64 device tensor [4] <- kept triangles, box pixels, block pairs, 64-bit triangles."""
    arr, nm = _meshes(meshes)
    c = camera(cam)
    _check(lib().tk_raster_stats(_ptr(link_xf), batch, arr, nm, ctypes.byref(c), _ptr(stats), _stream(stream)))


# ------------------------------------------------------------------ batched problems

class Batch:
    """Many independent problems driven by batched launches: a host array of
    tk_problem and its device table (written once by tk_batch_describe)."""

    def __init__(self, problems, device="cuda"):
        self.problems = (Problem * len(problems))(*problems)
        self.n = len(problems)
        nbytes = int(lib().tk_batch_table_bytes(self.n))
        if nbytes == 0:
            raise TkError(TK_ERR_INVALID_ARGUMENT, f"bad number of problems {self.n}")
        host = np.zeros(nbytes + 256, dtype=np.uint8)
        off = (-host.ctypes.data) % 256
        view = host[off:off + nbytes]
        _check(lib().tk_batch_describe(self.problems, self.n, view.ctypes.data_as(ctypes.c_void_p), nbytes))
        self.table = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        doff = (-self.table.data_ptr()) % 256
        self.table_view = self.table[doff:doff + nbytes]
        self.table_view.copy_(torch.from_numpy(view.copy()))

    def ask_eval(self, stream=None):
        _check(lib().tk_batch_ask_eval(self.problems, self.n, _ptr(self.table_view), _stream(stream)))

    def ask_eval_persistent(self, stream=None):
        """All problems' ask-eval in one persistent launch (per 128 problems)."""
        _check(lib().tk_batch_ask_eval_persistent(self.problems, self.n, _ptr(self.table_view), _stream(stream)))

    def tell(self, stream=None):
        _check(lib().tk_batch_tell(self.problems, self.n, _ptr(self.table_view), _stream(stream)))
