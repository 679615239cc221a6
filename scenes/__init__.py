"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module produces DATA only: a procedural instrument mesh, the kinematic
chain constants, pinhole cameras, seeded true poses, pixel-flip sets, occluder
rectangles and trajectories.  It holds none of the method's arithmetic (no
forward kinematics, no projection, no rasterisation, no CMA-ES); whoever needs
a rendered target renders it with their own implementation.

The paper's CAD mesh of the Large Needle Driver and its datasets are not
available, so the shapes stand in for them (paper Sec. III-A, Eq. for the
renderer input v_m; Sec. IV synthetic/real datasets: 640x480 and 700x493
masks, joint limits, 1000-frame trajectories).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 11404

# Sub-stream offsets added to a config's base seed.
SUB_POSE, SUB_FLIPS, SUB_OCCLUDER, SUB_CMAES, SUB_TRAJ = 0, 1, 2, 3, 4

LINK_SHAFT, LINK_WRIST, LINK_JAW_POS, LINK_JAW_NEG = 0, 1, 2, 3
N_LINKS = 4
N_PARAMS = 9  # alpha, beta, gamma, x, y, z, qhat1, qhat2, qhat3


@dataclasses.dataclass
class Mesh:
    vertices: np.ndarray   # [V,3] float32, metres, link frame of vertex_link
    triangles: np.ndarray  # [T,3] int32
    vertex_link: np.ndarray  # [V] uint8, non-decreasing
    shape: dict            # generator parameters

    @property
    def n_vertices(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def n_triangles(self) -> int:
        return int(self.triangles.shape[0])


@dataclasses.dataclass
class Chain:
    d_pitch_yaw: float          # distance wrist-pitch axis -> yaw axis along z (m)
    q_lb: np.ndarray            # [3] joint lower limits (rad)
    q_ub: np.ndarray            # [3] joint upper limits (rad)
    keypoints: np.ndarray       # [4,4] float: x, y, z (link frame, m), link id


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = float(np.float32(0.01))   # 1 cm, stored as the float32 value both sides use


# --------------------------------------------------------------------------
# Procedural instrument mesh
# --------------------------------------------------------------------------

def _quad_grid(p0, du, dv, nu, nv):
    """Vertices and triangles of a planar nu x nv grid p0 + i/nu*du + j/nv*dv."""
    p0, du, dv = (np.asarray(a, dtype=np.float64) for a in (p0, du, dv))
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nv + 1), indexing="ij")
    verts = p0 + (ii[..., None] / nu) * du + (jj[..., None] / nv) * dv
    verts = verts.reshape(-1, 3)
    idx = np.arange((nu + 1) * (nv + 1)).reshape(nu + 1, nv + 1)
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    tris = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)])
    return verts, tris


def _weld(verts, tris, tol=1e-9):
    """Merges vertices closer than tol (the same point reached along two face
    grids) into the first of them; returns (vertices, triangles)."""
    from scipy.spatial import cKDTree
    n = len(verts)
    rep = np.arange(n)
    for i, j in sorted(cKDTree(verts).query_pairs(tol)):
        ri, rj = rep[i], rep[j]
        while rep[ri] != ri:
            ri = rep[ri]
        while rep[rj] != rj:
            rj = rep[rj]
        rep[max(ri, rj)] = min(ri, rj)
    for i in range(n):
        r = i
        while rep[r] != r:
            r = rep[r]
        rep[i] = r
    keep = np.unique(rep)
    new_index = np.full(n, -1)
    new_index[keep] = np.arange(len(keep))
    return verts[keep], new_index[rep][tris]


def _tri_subdiv(p0, p1, p2, m):
    """Split triangle p0 p1 p2 into m*m congruent triangles."""
    p0, p1, p2 = (np.asarray(a, dtype=np.float64) for a in (p0, p1, p2))
    verts, index = [], {}
    for i in range(m + 1):
        for j in range(m + 1 - i):
            index[(i, j)] = len(verts)
            verts.append(p0 + (i / m) * (p1 - p0) + (j / m) * (p2 - p0))
    tris = []
    for i in range(m):
        for j in range(m - i):
            tris.append((index[(i, j)], index[(i + 1, j)], index[(i, j + 1)]))
            if j < m - i - 1:
                tris.append((index[(i + 1, j)], index[(i + 1, j + 1)], index[(i, j + 1)]))
    return np.array(verts), np.array(tris, dtype=np.int64)


def instrument_mesh(segments=32, rings=28, box_div=3, wedge_div=1,
                    jaw_scale=1.0, box_scale=1.0) -> Mesh:
    """Procedural stand-in for the Large Needle Driver.

    Link frames: the end-effector (robot) frame sits at the wrist-pitch axis
    with z pointing distally (paper Fig. 2 caption, Sec. III-A).
      * shaft (link 0): cylinder r = 4 mm on z in [-0.302, -0.002] closed by
        two end discs; `segments` around, `rings` interior rings ->
        2*segments*(rings+1) side tris + 2*segments cap tris.
      * wrist (link 1): box x, y in +-3.5 mm (x box_scale), z in [-0.002, 0.009];
        each face split box_div x box_div -> 12*box_div^2 tris.
      * jaws (links 2, 3): triangular prisms in the jaw frames, base half-width
        2.5 mm, length 14 mm (x jaw_scale), y in +-2 mm; jaw+ in x >= 0, jaw-
        mirrored -> 16*wedge_div^2 tris.
    Vertices are emitted sorted by link.  Each part is a closed surface with
    outward-consistent winding: its face grids share (welded) vertices, so
    every edge a->b of a triangle appears exactly as often as b->a.
    """
    parts = []  # (verts, tris, link)

    # shaft
    r0, z0, z1 = 0.004, -0.302, -0.002
    nz = rings + 2
    ang = 2.0 * math.pi * np.arange(segments) / segments
    zs = np.linspace(z0, z1, nz)
    verts = np.stack([np.repeat(np.cos(ang)[None, :] * r0, nz, 0),
                      np.repeat(np.sin(ang)[None, :] * r0, nz, 0),
                      np.repeat(zs[:, None], segments, 1)], -1).reshape(-1, 3)
    tris = []
    for i in range(nz - 1):
        for j in range(segments):
            a = i * segments + j
            b = i * segments + (j + 1) % segments
            c = (i + 1) * segments + (j + 1) % segments
            d = (i + 1) * segments + j
            tris.append((a, b, c))
            tris.append((a, c, d))
    # end discs: a fan about a centre vertex at each end, wound so that each
    # rim edge runs opposite to the side triangle sharing it
    lo, hi = len(verts), len(verts) + 1
    top = (nz - 1) * segments
    for j in range(segments):
        tris.append((lo, (j + 1) % segments, j))
        tris.append((hi, top + j, top + (j + 1) % segments))
    verts = np.concatenate([verts, [[0.0, 0.0, z0], [0.0, 0.0, z1]]])
    parts.append((verts, np.array(tris, dtype=np.int64), LINK_SHAFT))

    # wrist box
    h = 0.0035 * box_scale
    bz0, bz1 = -0.002, 0.009
    k = box_div
    faces = [
        ((-h, -h, bz0), (2 * h, 0, 0), (0, 2 * h, 0)),      # z = bz0
        ((-h, -h, bz1), (0, 2 * h, 0), (2 * h, 0, 0)),      # z = bz1
        ((-h, -h, bz0), (0, 0, bz1 - bz0), (2 * h, 0, 0)),  # y = -h
        ((-h, h, bz0), (2 * h, 0, 0), (0, 0, bz1 - bz0)),   # y = +h
        ((-h, -h, bz0), (0, 2 * h, 0), (0, 0, bz1 - bz0)),  # x = -h
        ((h, -h, bz0), (0, 0, bz1 - bz0), (0, 2 * h, 0)),   # x = +h
    ]
    bv, bt = [], []
    for p0, du, dv in faces:
        v, t = _quad_grid(p0, du, dv, k, k)
        bt.append(t + sum(len(x) for x in bv))
        bv.append(v)
    parts.append((*_weld(np.concatenate(bv), np.concatenate(bt)), LINK_WRIST))

    # jaws
    w = 0.0025 * jaw_scale
    L = 0.014 * jaw_scale
    hy = 0.002
    m = wedge_div
    for sign, link in ((1.0, LINK_JAW_POS), (-1.0, LINK_JAW_NEG)):
        A = np.array([0.0, 0.0]); B = np.array([sign * w, 0.0]); C = np.array([0.0, L])

        def xyz(p, y):
            return (p[0], y, p[1])
        wv, wt = [], []

        def add(v, t):
            wt.append(t + sum(len(x) for x in wv))
            wv.append(v)
        # two caps at y = -hy, +hy, wound opposite ways (each against the sides it meets)
        add(*_tri_subdiv(xyz(A, -hy), xyz(C, -hy), xyz(B, -hy), m))
        add(*_tri_subdiv(xyz(A, hy), xyz(B, hy), xyz(C, hy), m))
        # three rectangular sides
        for P, Q in ((A, B), (B, C), (C, A)):
            p0 = xyz(P, -hy)
            du = np.subtract(xyz(Q, -hy), p0)
            dv = (0.0, 2 * hy, 0.0)
            add(*_quad_grid(p0, du, dv, m, m))
        parts.append((*_weld(np.concatenate(wv), np.concatenate(wt)), link))

    all_v, all_t, all_l = [], [], []
    off = 0
    for v, t, link in parts:
        all_v.append(v)
        all_t.append(t + off)
        all_l.append(np.full(len(v), link, dtype=np.uint8))
        off += len(v)
    return Mesh(np.concatenate(all_v).astype(np.float32),
                np.concatenate(all_t).astype(np.int32),
                np.concatenate(all_l),
                dict(segments=segments, rings=rings, box_div=box_div, wedge_div=wedge_div,
                     jaw_scale=jaw_scale, box_scale=box_scale))


def mesh_for_triangles(n_tris: int, jaw_scale=1.0, box_scale=1.0) -> Mesh:
    """Procedural mesh with a triangle count close to n_tris (exact count in .n_triangles)."""
    if n_tris < 8000:
        s, k, m = 32, 3, 1
    else:
        s, k, m = 64, 6, 4
    rest = n_tris - 12 * k * k - 16 * m * m - 2 * s
    rings = max(0, int(round(rest / (2 * s))) - 1)
    return instrument_mesh(s, rings, k, m, jaw_scale, box_scale)


def chain(jaw_scale=1.0) -> Chain:
    """Chain constants matching instrument_mesh (joint limits: q1, q2 in
    [-pi/2, pi/2], jaw q3 in [0, pi/2]; keypoints: shaft end, yaw centre, two
    jaw tips)."""
    d = 0.009
    L = 0.014 * jaw_scale
    kp = np.array([[0.0, 0.0, -0.002, LINK_SHAFT],
                   [0.0, 0.0, d, LINK_WRIST],
                   [0.0, 0.0, L, LINK_JAW_POS],
                   [0.0, 0.0, L, LINK_JAW_NEG]], dtype=np.float64)
    return Chain(d, np.array([-math.pi / 2, -math.pi / 2, 0.0]),
                 np.array([math.pi / 2, math.pi / 2, math.pi / 2]), kp)


def camera(width: int, height: int, f: float | None = None) -> Camera:
    """Pinhole camera, principal point at the image centre, f = 1.25*W unless given."""
    if f is None:
        f = 1.25 * width
    return Camera(float(f), float(f), width / 2.0, height / 2.0, int(width), int(height))


# --------------------------------------------------------------------------
# Poses, targets, trajectories
# --------------------------------------------------------------------------

def rng_for(config_index: int, sub: int) -> np.random.Generator:
    return np.random.default_rng(BASE_SEED + config_index + 1000 * sub)


def true_pose(rng: np.random.Generator, cam: Camera) -> np.ndarray:
    """One seeded physical parameter vector (alpha, beta, gamma, x, y, z, qhat1..3).

    Chosen by bounds, without rendering: the wrist sits at depth 8-15 cm inside
    the central half of the field of view; alpha near pi and |gamma| <= 0.8
    tilt the shaft 20-60 deg away from the camera so every vertex stays at
    least ~5 cm deep; beta is uniform; joints are drawn in the unconstrained
    coordinate.
    """
    z = rng.uniform(0.08, 0.15)
    x = z * rng.uniform(-0.25, 0.25) * cam.width / cam.fx
    y = z * rng.uniform(-0.25, 0.25) * cam.height / cam.fy
    alpha = math.pi + rng.choice([-1.0, 1.0]) * rng.uniform(0.35, 0.8)
    gamma = rng.choice([-1.0, 1.0]) * rng.uniform(0.2, 0.8)
    beta = rng.uniform(-math.pi, math.pi)
    qh1 = rng.uniform(-0.8, 0.8)
    qh2 = rng.uniform(-0.8, 0.8)
    qh3 = rng.uniform(0.3, 0.8)
    return np.array([alpha, beta, gamma, x, y, z, qh1, qh2, qh3], dtype=np.float64)


#: Normalisation scales s in theta = o + s * x (rad, rad, rad, m, m, m, rad, rad, rad).
DEFAULT_SCALE = np.array([0.05, 0.05, 0.05, 0.005, 0.005, 0.005, 0.1, 0.1, 0.1])


def trajectory(rng: np.random.Generator, cam: Camera, n_frames: int) -> np.ndarray:
    """Smooth seeded trajectory [n_frames, 9]: per frame the translation moves
    exactly 1 mm and the look-at angles exactly 0.5 deg (Euclidean in angle
    space) along slowly turning seeded directions; the joints follow seeded
    sinusoids in the unconstrained coordinate."""
    th = true_pose(rng, cam)
    out = np.empty((n_frames, N_PARAMS))
    dir_t = rng.normal(size=3)
    dir_r = rng.normal(size=3)
    ph = rng.uniform(0, 2 * math.pi, size=3)
    fr = rng.uniform(0.02, 0.06, size=3)
    amp = np.array([0.5, 0.5, 0.2])
    mid = np.array([0.0, 0.0, 0.55])
    for t in range(n_frames):
        out[t] = th
        out[t, 6:9] = mid + amp * np.sin(fr * t + ph)
        dir_t = dir_t + 0.3 * rng.normal(size=3)
        dir_r = dir_r + 0.3 * rng.normal(size=3)
        # keep the wrist inside the depth band and the shaft tilted away
        if th[5] > 0.14:
            dir_t[2] = -abs(dir_t[2])
        if th[5] < 0.09:
            dir_t[2] = abs(dir_t[2])
        th = th.copy()
        th[3:6] += 0.001 * dir_t / np.linalg.norm(dir_t)
        th[0:3] += math.radians(0.5) * dir_r / np.linalg.norm(dir_r)
        th[0] = min(max(th[0], math.pi - 0.8), math.pi + 0.8)
        th[2] = min(max(th[2], -0.8), 0.8)
    return out


def hermite_trajectory(rng: np.random.Generator, cam: Camera, n_frames: int, n_waypoints: int = 20) -> np.ndarray:
    """Seeded trajectory [n_frames, 9] in the manner of the paper's synthetic
    set (Sec. IV, synthetic dataset): feasible waypoints (a bounded random walk
    from a true pose: look-at angles, translation inside the view and the
    depth band, joints across their range) joined by cubic Hermite splines
    with Catmull-Rom tangents, plus temporally correlated Ornstein-Uhlenbeck
    noise, then smoothed by a zero-phase first-order low-pass filter."""
    w = np.empty((n_waypoints, N_PARAMS))
    w[0] = true_pose(rng, cam)
    side = 1.0 if w[0, 0] > math.pi else -1.0
    for k in range(1, n_waypoints):
        p = w[k - 1].copy()
        p[0:3] += rng.uniform(-0.15, 0.15, 3)
        p[3:6] += rng.uniform(-0.008, 0.008, 3)
        p[6:9] = [rng.uniform(-0.8, 0.8), rng.uniform(-0.8, 0.8), rng.uniform(0.3, 0.8)]
        p[0] = math.pi + side * min(max(side * (p[0] - math.pi), 0.35), 0.8)
        p[2] = min(max(p[2], -0.8), 0.8)
        p[5] = min(max(p[5], 0.08), 0.15)
        p[3] = min(max(p[3], -0.25 * p[5] * cam.width / cam.fx), 0.25 * p[5] * cam.width / cam.fx)
        p[4] = min(max(p[4], -0.25 * p[5] * cam.height / cam.fy), 0.25 * p[5] * cam.height / cam.fy)
        w[k] = p
    tang = np.empty_like(w)
    tang[1:-1] = 0.5 * (w[2:] - w[:-2])
    tang[0], tang[-1] = w[1] - w[0], w[-1] - w[-2]
    out = np.empty((n_frames, N_PARAMS))
    for t in range(n_frames):
        sp = t * (n_waypoints - 1) / max(n_frames - 1, 1)
        k = min(int(sp), n_waypoints - 2)
        u = sp - k
        h00, h10 = 2 * u ** 3 - 3 * u ** 2 + 1, u ** 3 - 2 * u ** 2 + u
        h01, h11 = -2 * u ** 3 + 3 * u ** 2, u ** 3 - u ** 2
        out[t] = h00 * w[k] + h10 * tang[k] + h01 * w[k + 1] + h11 * tang[k + 1]
    # Ornstein-Uhlenbeck noise (mean reversion 0.1 per frame)
    amp = np.array([0.002, 0.002, 0.002, 0.0002, 0.0002, 0.0002, 0.005, 0.005, 0.005])
    ou = np.zeros(N_PARAMS)
    for t in range(n_frames):
        ou = ou - 0.1 * ou + amp * rng.normal(size=N_PARAMS)
        out[t] += ou
    # zero-phase low-pass: first-order smoothing forward, then backward
    a = 0.3
    for order in (range(1, n_frames), range(n_frames - 2, -1, -1)):
        step = 1 if order.step == 1 else -1
        for t in order:
            out[t] = a * out[t] + (1 - a) * out[t - step]
    return out


def perturb_mask(rng: np.random.Generator, image: np.ndarray) -> np.ndarray:
    """Segmentation errors in the manner of the paper's synthetic set: a random
    dilation or erosion (1-2 steps of a 3x3 element, or none), then 2-6 disc
    blobs of radius 2-5 px centred on boundary pixels, each added or cut."""
    from scipy import ndimage

    img = np.asarray(image, dtype=bool)
    op = rng.choice(3, p=[0.4, 0.4, 0.2])
    it = int(rng.integers(1, 3))
    if op == 0:
        img = ndimage.binary_dilation(img, iterations=it)
    elif op == 1:
        img = ndimage.binary_erosion(img, iterations=it)
    edge = np.argwhere(img ^ ndimage.binary_erosion(img))
    if len(edge):
        yy, xx = np.mgrid[0:img.shape[0], 0:img.shape[1]]
        for _ in range(int(rng.integers(2, 7))):
            cy, cx = edge[rng.integers(len(edge))]
            r = rng.uniform(2.0, 5.0)
            disc = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
            img = img | disc if rng.random() < 0.5 else img & ~disc
    return img


# --------------------------------------------------------------------------
# Mask layout helpers (bit ly*8+lx of word [y/8][x/8]) and corruptions
# --------------------------------------------------------------------------

def mask_words_shape(width: int, height: int) -> tuple[int, int]:
    return ((height + 7) // 8, (width + 7) // 8)


def words_to_image(words: np.ndarray, width: int, height: int) -> np.ndarray:
    """[..., by, bx] uint64 words -> [..., H, W] bool image."""
    words = np.asarray(words, dtype=np.uint64)
    by, bx = mask_words_shape(width, height)
    lead = words.shape[:-2]
    bits = ((words[..., None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(bool)
    bits = bits.reshape(*lead, by, bx, 8, 8)            # ly, lx
    img = np.moveaxis(bits, -2, -3).reshape(*lead, by * 8, bx * 8)
    return img[..., :height, :width]


def image_to_words(img: np.ndarray) -> np.ndarray:
    """[..., H, W] bool -> [..., ceil(H/8), ceil(W/8)] uint64 words (padding bits zero)."""
    img = np.asarray(img, dtype=bool)
    *lead, H, W = img.shape
    by, bx = mask_words_shape(W, H)
    pad = np.zeros((*lead, by * 8, bx * 8), dtype=bool)
    pad[..., :H, :W] = img
    t = pad.reshape(*lead, by, 8, bx, 8)
    t = np.moveaxis(t, -3, -2)                          # by, bx, ly, lx
    t = t.reshape(*lead, by, bx, 64).astype(np.uint64)
    return (t << np.arange(64, dtype=np.uint64)).sum(-1, dtype=np.uint64)


def flip_indices(rng: np.random.Generator, width: int, height: int, fraction=0.01) -> np.ndarray:
    """Exactly round(fraction*W*H) distinct seeded pixel indices (y*W + x)."""
    n = int(round(fraction * width * height))
    return rng.choice(width * height, size=n, replace=False).astype(np.int64)


def apply_flips(words: np.ndarray, width: int, height: int, idx: np.ndarray) -> np.ndarray:
    """XOR-flip the given pixels of a word mask (returns a copy)."""
    out = np.array(words, dtype=np.uint64, copy=True)
    y, x = np.divmod(np.asarray(idx, dtype=np.int64), width)
    bit = ((y % 8) * 8 + (x % 8)).astype(np.uint64)
    flat = out.reshape(-1)
    widx = (y // 8) * ((width + 7) // 8) + x // 8
    for w, b in zip(widx, bit):
        flat[w] ^= np.uint64(1) << b
    return out


def occluder_rect(img: np.ndarray, rng: np.random.Generator, lo=0.1, hi=0.3):
    """Axis-aligned rectangle (x0, y0, x1, y1), exclusive ends, covering a
    fraction phi ~ U[lo, hi] of the silhouette's pixels: a square grown around
    a random silhouette pixel until it holds at least phi of them."""
    img = np.asarray(img, dtype=bool)
    ys, xs = np.nonzero(img)
    total = len(ys)
    phi = rng.uniform(lo, hi)
    if total == 0:
        return (0, 0, 0, 0), phi
    i = rng.integers(total)
    cy, cx = int(ys[i]), int(xs[i])
    H, W = img.shape
    csum = np.pad(img.astype(np.int64).cumsum(0).cumsum(1), ((1, 0), (1, 0)))
    r = 0
    while True:
        x0, x1 = max(cx - r, 0), min(cx + r + 1, W)
        y0, y1 = max(cy - r, 0), min(cy + r + 1, H)
        inside = csum[y1, x1] - csum[y0, x1] - csum[y1, x0] + csum[y0, x0]
        if inside >= phi * total or (x0 == 0 and y0 == 0 and x1 == W and y1 == H):
            return (x0, y0, x1, y1), phi
        r += 1


def apply_occluder(img: np.ndarray, rect) -> np.ndarray:
    x0, y0, x1, y1 = rect
    out = np.array(img, dtype=bool, copy=True)
    out[..., y0:y1, x0:x1] = False
    return out


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

# Noise of the temporal filter for the seeded track640 trajectories, per frame
# (dt = 1 frame), in the filter's coordinates (look-at angles [rad],
# translation [m], joint angles [rad]).  meas_std: robust spread (1.4826 x
# median absolute error) of the raw per-frame CMA-ES estimates; vel_std: half
# the RMS frame-to-frame velocity change of the trajectories; pos_std: a tenth
# of vel_std.  Medians over trajectories 1, 12, 13 and 14 of this generator.
FILTER_TRACK = dict(
    dt=1.0,
    meas_std=np.array([7.7e-4, 3.3e-4, 5.2e-4, 7.7e-6, 1.0e-5, 8.1e-5, 7.2e-4, 5.6e-4, 3.3e-4]),
    vel_std=np.array([4.1e-4, 3.6e-4, 2.5e-4, 3.4e-5, 3.4e-5, 5.7e-5, 3.1e-4, 5.3e-4, 1.5e-4]),
    pos_std=np.array([4.1e-5, 3.6e-5, 2.5e-5, 3.4e-6, 3.4e-6, 5.7e-6, 3.1e-5, 5.3e-5, 1.5e-5]),
)


def workload(name: str) -> dict:
    """Shapes of the named synthetic workloads: meshes, chains, camera, lambda,
    generations per frame, frames, workload index (seed offset) and the number
    of diagonal covariance blocks."""
    if name == "small":          # 2k tris, 320x240, f=400, lambda=16, 20 gens
        return dict(mesh=instrument_mesh(32, 28, 3, 1), cam=camera(320, 240, 400.0),
                    lam=16, gens=20, frames=1, index=0)
    if name == "track640":       # 20k tris, 640x480, lambda=256, 30 gens x 100 frames
        return dict(mesh=instrument_mesh(64, 150, 6, 4), cam=camera(640, 480),
                    lam=256, gens=30, frames=100, index=1, filter=FILTER_TRACK)
    if name == "bimanual960":    # two uneven instruments (20144 + 35388 tris), 960x540, lambda=512, 18-D
        meshes = [instrument_mesh(64, 150, 6, 4), instrument_mesh(100, 170, 7, 5, jaw_scale=1.3, box_scale=1.2)]
        return dict(meshes=meshes, mesh=meshes[0], chains=[chain(), chain(jaw_scale=1.3)], cam=camera(960, 540),
                    lam=512, gens=30, frames=1, index=2, n_blocks=2)
    if name == "synth700":       # the paper's synthetic-set protocol: 700x493, N = 70, 3 iterations per
        # frame with raised learning rates (c_mu x2, sigma0 0.5: a reading, the paper gives no values),
        # 1000-frame Hermite/OU trajectory, dilation / erosion / edge-blob masks, the render loss (MSE +
        # appearance) plus the two-tip keypoint term in pixels (weights: a reading, the paper gives none)
        return dict(mesh=instrument_mesh(64, 150, 6, 4), cam=camera(700, 493), lam=70, gens=3, frames=1000,
                    index=5, filter=FILTER_TRACK, sigma0=0.5, c_m_scale=1.0, c_mu_scale=2.0,
                    lambda_app=1.0, lambda_kp=10.0, tau=2.0)
    if name == "soft640":        # differentiable form: 49744 tris, 640x480, 256 candidates, sigma = 1 px
        return dict(mesh=instrument_mesh(100, 240, 8, 6), cam=camera(640, 480), lam=256, gens=30, frames=1,
                    index=4, sigma=1.0)
    raise KeyError(name)


BATCH_RESOLUTIONS = ((320, 240), (640, 480), (960, 540), (1280, 720))
BATCH_LAMBDAS = (64, 128, 256, 512, 1024)


def batch_problem_shapes(count: int = 64, seed_index: int = 3) -> list[dict]:
    """Shapes of the batched-solves workload: problem p has resolution
    BATCH_RESOLUTIONS[p % 4], lambda = BATCH_LAMBDAS[(p // 4) % 5] and a mesh of
    about T = round(2000 * 25**u) triangles, u ~ U[0, 1] seeded (log-uniform
    between 2k and 50k): an instrument with 32 (T < 8000) or 64 shaft segments
    and as many rings as bring it closest to T."""
    rng = rng_for(seed_index, SUB_POSE)
    out = []
    for p in range(count):
        W, H = BATCH_RESOLUTIONS[p % 4]
        target_t = int(round(2000 * 25 ** rng.uniform()))
        seg = 32 if target_t < 8000 else 64
        rings = max(1, int(round((target_t - 124) / (2 * seg))) - 1)
        out.append(dict(width=W, height=H, lam=BATCH_LAMBDAS[(p // 4) % 5], segments=seg, rings=rings,
                        target_triangles=target_t))
    return out
