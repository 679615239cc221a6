// Soft (differentiable) silhouette of the candidates and its backward pass.
//
// The soft silhouette stands in for the renderer S = R(K(Pi(T_r^c T_m^r(q)
// v_m))) of Sec. III-A.2 where a gradient is wanted; its loss is the
// squared-error term of Eq. (6) summed over the pixels:
//   d_j(p)    signed Euclidean distance from the pixel centre to the boundary
//             of face j (positive inside), FP32 projected corners, no snapping;
//   prob_j(p) = (sig(d_j / sigma) - s0) / (1 - s0) for d_j >= -10 sigma, else
//             0, s0 = sig(-10) (the logistic shifted to reach 0 at the cutoff,
//             so that the image is continuous in theta);
//   S(p)      = 1 - prod_j (1 - prob_j(p)) over the faces of every arm;
//   L         = sum_p (S(p) - M(p))^2.
// Faces with a corner in front of z_near or with zero projected area are left
// out.  With log(1 - prob_j) = softplus(-10) - softplus(d_j / sigma), the
// forward pass sums these logs per pixel and the backward pass needs, per
// (pixel, face), only dL/dd_j = G(p) sig(d_j / sigma) with
// G(p) = 2 (S - M)(1 - S) / sigma.
//
// Forward (pixel-major): corners are projected once per candidate, face
// records carry the corners, inverse edge lengths, orientation and the pixel
// range of the 10-sigma band; one workgroup per candidate bins the faces into
// 8x8-pixel tiles (LDS counters; a face covering more than 32 tiles goes to a
// per-candidate list that every tile scans); one wave per tile sums the logs
// of its pixels over the tile's faces in 64-bit fixed point (2^-32), so the
// order of the lists does not change a bit of the result.
// Backward (face-major): one lane per face walks the pixels of its band,
// accumulates dL/d(corner) from G, projects it through the pinhole Jacobian
// into dL/dM_l (the 3x4 link transforms), reduced per workgroup in a fixed
// order; a last kernel sums the workgroups in order and applies the Jacobian
// of the forward kinematics (FP64, cosine joint map included).
#include <cmath>
#include <cstring>

#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kSoftTile = 8;               // 8 x 8 pixels per tile, one wave
constexpr int kSoftMaxTiles = 32;          // tiles per face in the tile lists
constexpr int kSoftMaxTileCount = 16384;   // tiles per image (LDS counters)
constexpr int kSoftBinThreads = 1024;
constexpr int kSoftFaceBlock = 256;        // threads per backward workgroup
constexpr int kSoftFaceLanes = 8;          // lanes per face in the backward pass
constexpr int kSoftFacesPerBlock = kSoftFaceBlock / kSoftFaceLanes;
           // waves per tile in the forward pass
constexpr int kSoftWideBin = 64;           // from this batch on, one binning workgroup per candidate
constexpr int kSoftBinGroups = 32;         // below it, binning workgroups per candidate
constexpr int kSoftFwdChunkSmall = 64;     // faces of a tile list per forward work item, batch < kSoftWideBin
constexpr int kSoftFwdChunkWide = 1024;    // the same from kSoftWideBin candidates on
constexpr int kSoftReduceGroups = 16;      // workgroups summing the backward partials of one candidate
constexpr int kSoftGrad = 48;              // dL/dM: 4 links x 12 entries
constexpr double kFixScale = 4294967296.0; // 2^32
constexpr float kBand = 10.0f;             // the band is d >= -10 sigma

struct FaceRec {              // 48 bytes
    float u[3], v[3];         // projected corners
    float il[3];              // 1 / squared length of edge e (corner e -> e+1); 0 for a point
    float orient;             // sign of the projected area, 0 = face left out
    int16_t x0, x1, y0, y1;   // pixels of the band, clamped to the image (x0 > x1: none)
};
static_assert(sizeof(FaceRec) == 48, "face record is 48 bytes");

struct SoftLayout {
    size_t verts, faces, tile_off, tile_cnt, tile_tot, chunks, chunk_n, facc, done, lists, big, big_n, G, tloss, part,
        gsum, total;
    int32_t tiles_x, tiles_y, n_tiles, n_blocks, chunk_cap, fwd_chunk;
};

struct SoftArgs {
    MeshSet ms;
    CamK cam;
    int32_t face_offset[kMaxArms];     // first face of each arm in the concatenated list
    int32_t block_offset[kMaxArms];    // first backward workgroup of each arm
    int32_t total_faces, batch;
    float sigma, inv_sigma;
    int32_t tiles_x, tiles_y, n_tiles, n_blocks, chunk_cap, fwd_chunk;
    // workspace
    float4* verts;        // [batch][V]
    FaceRec* faces;       // [batch][F]
    int32_t* tile_off;    // [batch][n_tiles + 1]
    int32_t* tile_cnt;    // [batch][kSoftBinGroups][n_tiles] each binning workgroup's first slot in a tile list
    int32_t* tile_tot;    // [batch][n_tiles] list lengths summed by the binning workgroups (both: batch < kSoftWideBin)
    int2* chunks;         // [batch][chunk_cap] forward work items (tile, k): faces k * fwd_chunk... of its list
    int32_t* chunk_n;     // [batch] work items
    long long* facc;      // [batch][n_tiles][64] fixed-point sums of tiles split over several items
    int32_t* done;        // [batch][n_tiles] items of a split tile finished
    int32_t* lists;       // [batch][F * kSoftMaxTiles]
    int32_t* big;         // [batch][F]
    int32_t* big_n;       // [batch]
    float* G;             // [batch][H * W]
    double* tloss;        // [batch][n_tiles]
    float* part;          // [batch][n_blocks][kSoftGrad]
    double* gsum;         // [batch][kSoftReduceGroups][kMaxArms][kSoftGrad] sums of slices of the partials
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

SoftLayout soft_layout(int32_t batch, const MeshSet& ms, int32_t total_faces, int32_t W, int32_t H,
                       const int32_t* faces_per_arm) {
    SoftLayout L;
    L.tiles_x = (W + kSoftTile - 1) / kSoftTile;
    L.tiles_y = (H + kSoftTile - 1) / kSoftTile;
    L.n_tiles = L.tiles_x * L.tiles_y;
    L.n_blocks = 0;
    // each tile: one work item, or one per fwd_chunk faces of a longer list
    L.fwd_chunk = batch < kSoftWideBin ? kSoftFwdChunkSmall : kSoftFwdChunkWide;
    L.chunk_cap = int32_t(L.n_tiles + (size_t(total_faces) * kSoftMaxTiles + L.fwd_chunk - 1) / L.fwd_chunk);
    for (int a = 0; a < ms.n_meshes; a++) L.n_blocks += (faces_per_arm[a] + kSoftFacesPerBlock - 1) / kSoftFacesPerBlock;
    const size_t B = size_t(batch), V = size_t(ms.total_vertices), F = size_t(total_faces);
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t r = o;
        o = align256(o + bytes);
        return r;
    };
    L.verts = take(B * V * sizeof(float4));
    L.faces = take(B * F * sizeof(FaceRec));
    L.tile_off = take(B * size_t(L.n_tiles + 1) * sizeof(int32_t));
    L.tile_cnt = take(batch < kSoftWideBin ? B * kSoftBinGroups * size_t(L.n_tiles) * sizeof(int32_t) : 0);
    L.tile_tot = take(batch < kSoftWideBin ? B * size_t(L.n_tiles) * sizeof(int32_t) : 0);
    L.chunks = take(B * size_t(L.chunk_cap) * sizeof(int2));
    L.chunk_n = take(B * sizeof(int32_t));
    L.facc = take(B * size_t(L.n_tiles) * 64 * sizeof(long long));
    L.done = take(B * size_t(L.n_tiles) * sizeof(int32_t));
    L.lists = take(B * F * kSoftMaxTiles * sizeof(int32_t));
    L.big = take(B * F * sizeof(int32_t));
    L.big_n = take(B * sizeof(int32_t));
    L.G = take(B * size_t(W) * size_t(H) * sizeof(float));
    L.tloss = take(B * size_t(L.n_tiles) * sizeof(double));
    L.part = take(B * size_t(L.n_blocks) * kSoftGrad * sizeof(float));
    L.gsum = take(B * kSoftReduceGroups * kMaxArms * kSoftGrad * sizeof(double));
    L.total = o;
    return L;
}

// ---------------------------------------------------------------- device helpers

// Arm of a concatenated vertex / face index (at most two arms).
__device__ __forceinline__ int arm_of(int32_t g, int32_t second_start, int32_t n_meshes) {
    return (n_meshes > 1 && g >= second_start) ? 1 : 0;
}

// softplus(x) = log(1 + e^x), stable for either sign
__device__ __forceinline__ float softplus_f(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }

// Signed distance of the pixel centre (px, py) to the face boundary (positive
// inside): the smallest point-to-segment distance over the three edges (the
// first edge on a tie), with the nearest edge's corners (ia, ib), the
// parameter t of its closest point and the unit vector (nx, ny) from that
// point to the pixel; sg = +1 inside, -1 outside.
struct EdgeHit {
    float d, t, nx, ny, sg;
    int ia;
};
__device__ __forceinline__ EdgeHit face_distance(const FaceRec& f, float px, float py) {
    float best = INFINITY, bt = 0.0f, brx = 0.0f, bry = 0.0f;
    int bia = 0;
    bool in_all = true;
#pragma unroll
    for (int e = 0; e < 3; e++) {
        const int b = e == 2 ? 0 : e + 1;
        const float ex = f.u[b] - f.u[e], ey = f.v[b] - f.v[e];
        const float wx = px - f.u[e], wy = py - f.v[e];
        float t = (wx * ex + wy * ey) * f.il[e];
        t = fminf(fmaxf(t, 0.0f), 1.0f);
        const float rx = wx - t * ex, ry = wy - t * ey;
        const float d2 = rx * rx + ry * ry;
        if (d2 < best) {
            best = d2;
            bt = t;
            brx = rx;
            bry = ry;
            bia = e;
        }
        const float cr = ex * wy - ey * wx;
        in_all = in_all && cr * f.orient >= 0.0f;
    }
    EdgeHit h;
    const float dist = sqrtf(best);
    h.d = in_all ? dist : -dist;
    h.sg = in_all ? 1.0f : -1.0f;
    h.t = bt;
    h.nx = dist > 0.0f ? brx / dist : 0.0f;
    h.ny = dist > 0.0f ? bry / dist : 0.0f;
    h.ia = bia;
    return h;
}

// ---------------------------------------------------------------- forward kernels

__global__ __launch_bounds__(256) void soft_vert_kernel(const float* __restrict__ link_xf, SoftArgs a) {
    const int32_t gv = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (gv >= a.ms.total_vertices) return;
    const int arm = arm_of(gv, a.ms.m[1].vertex_offset, a.ms.n_meshes);
    const MeshK m = arm == 0 ? a.ms.m[0] : a.ms.m[1];
    const int32_t vi = gv - m.vertex_offset;
    const int l = m.vertex_link[vi];
    const float* M = link_xf + ((size_t(b) * a.ms.n_meshes + arm) * 4 + l) * 12;
    const float vx = m.vertices[3 * vi], vy = m.vertices[3 * vi + 1], vz = m.vertices[3 * vi + 2];
    const float X = M[0] * vx + M[1] * vy + M[2] * vz + M[3];
    const float Y = M[4] * vx + M[5] * vy + M[6] * vz + M[7];
    const float Z = M[8] * vx + M[9] * vy + M[10] * vz + M[11];
    const float u = a.cam.fx * (X / Z) + a.cam.cx;
    const float v = a.cam.fy * (Y / Z) + a.cam.cy;
    const bool ok = Z >= a.cam.z_near && isfinite(u) && isfinite(v);
    a.verts[size_t(b) * a.ms.total_vertices + gv] = make_float4(u, v, Z, ok ? 1.0f : 0.0f);
}

__global__ __launch_bounds__(256) void soft_face_kernel(SoftArgs a) {
    if (a.tile_tot) {   // clear what the multi-workgroup binning accumulates
        const int b = blockIdx.y;
        if (blockIdx.x == 0 && threadIdx.x == 0) a.big_n[b] = 0;
        for (int t = blockIdx.x * 256 + threadIdx.x; t < a.n_tiles; t += gridDim.x * 256) a.tile_tot[size_t(b) * a.n_tiles + t] = 0;
    }
    const int32_t gf = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (gf >= a.total_faces) return;
    const int arm = arm_of(gf, a.face_offset[1], a.ms.n_meshes);
    const MeshK m = arm == 0 ? a.ms.m[0] : a.ms.m[1];
    const int32_t lf = gf - (arm == 0 ? a.face_offset[0] : a.face_offset[1]);
    const float4* V = a.verts + size_t(b) * a.ms.total_vertices + m.vertex_offset;
    FaceRec r;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const float4 p = V[m.triangles[3 * lf + c]];
        r.u[c] = p.x;
        r.v[c] = p.y;
        ok = ok && p.w != 0.0f;
    }
    const float area = (r.u[1] - r.u[0]) * (r.v[2] - r.v[0]) - (r.v[1] - r.v[0]) * (r.u[2] - r.u[0]);
    ok = ok && area != 0.0f && isfinite(area);
#pragma unroll
    for (int e = 0; e < 3; e++) {
        const int n = e == 2 ? 0 : e + 1;
        const float ex = r.u[n] - r.u[e], ey = r.v[n] - r.v[e];
        const float len2 = ex * ex + ey * ey;
        r.il[e] = len2 > 0.0f ? 1.0f / len2 : 0.0f;
    }
    r.orient = ok ? (area > 0.0f ? 1.0f : -1.0f) : 0.0f;
    const float hw = kBand * a.sigma;
    const float umin = fminf(fminf(r.u[0], r.u[1]), r.u[2]), umax = fmaxf(fmaxf(r.u[0], r.u[1]), r.u[2]);
    const float vmin = fminf(fminf(r.v[0], r.v[1]), r.v[2]), vmax = fmaxf(fmaxf(r.v[0], r.v[1]), r.v[2]);
    // pixel x takes part when its centre x + 0.5 lies in [umin - hw, umax + hw]
    const float fx0 = fmaxf(ceilf(umin - hw - 0.5f), 0.0f), fx1 = fminf(floorf(umax + hw - 0.5f), float(a.cam.width - 1));
    const float fy0 = fmaxf(ceilf(vmin - hw - 0.5f), 0.0f), fy1 = fminf(floorf(vmax + hw - 0.5f), float(a.cam.height - 1));
    if (ok && fx0 <= fx1 && fy0 <= fy1) {
        r.x0 = int16_t(fx0);
        r.x1 = int16_t(fx1);
        r.y0 = int16_t(fy0);
        r.y1 = int16_t(fy1);
    } else {
        r.x0 = 1;
        r.x1 = 0;
        r.y0 = 1;
        r.y1 = 0;
        r.orient = 0.0f;
    }
    a.faces[size_t(b) * a.total_faces + gf] = r;
}

// Binning: one workgroup per candidate, tile counters in LDS.
__global__ __launch_bounds__(kSoftBinThreads) void soft_bin_kernel(SoftArgs a) {
    __shared__ int32_t s_cnt[kSoftMaxTileCount];
    __shared__ int32_t s_part[kSoftBinThreads];
    __shared__ int32_t s_big;
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = a.n_tiles;
    const FaceRec* faces = a.faces + size_t(b) * a.total_faces;
    int32_t* lists = a.lists + size_t(b) * a.total_faces * kSoftMaxTiles;
    int32_t* big = a.big + size_t(b) * a.total_faces;
    for (int t = tid; t < nt; t += kSoftBinThreads) s_cnt[t] = 0;
    if (tid == 0) s_big = 0;
    __syncthreads();
    for (int32_t f = tid; f < a.total_faces; f += kSoftBinThreads) {
        const FaceRec r = faces[f];
        if (r.orient == 0.0f) continue;
        const int tx0 = r.x0 / kSoftTile, tx1 = r.x1 / kSoftTile, ty0 = r.y0 / kSoftTile, ty1 = r.y1 / kSoftTile;
        if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) > kSoftMaxTiles) {
            big[atomicAdd(&s_big, 1)] = f;
            continue;
        }
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) atomicAdd(&s_cnt[ty * a.tiles_x + tx], 1);
    }
    __syncthreads();
    // exclusive scan of the counts: contiguous chunks per thread, then the chunk sums
    const int chunk = (nt + kSoftBinThreads - 1) / kSoftBinThreads;
    const int c0 = min(tid * chunk, nt), c1 = min(c0 + chunk, nt);
    int32_t sum = 0;
    for (int t = c0; t < c1; t++) sum += s_cnt[t];
    s_part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kSoftBinThreads; off <<= 1) {
        const int32_t v = tid >= off ? s_part[tid - off] : 0;
        __syncthreads();
        s_part[tid] += v;
        __syncthreads();
    }
    int32_t run = s_part[tid] - sum;
    int32_t* off_out = a.tile_off + size_t(b) * (nt + 1);
    for (int t = c0; t < c1; t++) {
        const int32_t c = s_cnt[t];
        off_out[t] = run;
        s_cnt[t] = run;          // fill cursor
        run += c;
    }
    if (tid == kSoftBinThreads - 1) off_out[nt] = s_part[tid];
    if (tid == 0) a.big_n[b] = s_big;
    __syncthreads();
    for (int32_t f = tid; f < a.total_faces; f += kSoftBinThreads) {
        const FaceRec r = faces[f];
        if (r.orient == 0.0f) continue;
        const int tx0 = r.x0 / kSoftTile, tx1 = r.x1 / kSoftTile, ty0 = r.y0 / kSoftTile, ty1 = r.y1 / kSoftTile;
        if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) > kSoftMaxTiles) continue;
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) lists[atomicAdd(&s_cnt[ty * a.tiles_x + tx], 1)] = f;
    }
}

// Binning across workgroups for small batches (the single-workgroup form
// above leaves most of the chip idle then): workgroup g of a candidate counts
// the faces g * 256 + tid + k * kSoftBinGroups * 256 per tile in LDS and
// reserves that many slots of each tile it touches by one atomic add on the
// tile's total, which returns its first slot inside the tile's list; the plan
// pass turns the totals into list offsets; the fill pass repeats the count with
// LDS cursors from offset + first slot.  The order of the faces inside a tile
// list depends on the order of those atomics; the forward pass sums integers,
// so no result depends on it.  The face kernel clears big_n and the totals.
__device__ __forceinline__ bool face_tiles(const FaceRec& r, int& tx0, int& tx1, int& ty0, int& ty1) {
    tx0 = r.x0 / kSoftTile;
    tx1 = r.x1 / kSoftTile;
    ty0 = r.y0 / kSoftTile;
    ty1 = r.y1 / kSoftTile;
    return (tx1 - tx0 + 1) * (ty1 - ty0 + 1) <= kSoftMaxTiles;
}

__global__ __launch_bounds__(256) void soft_bin_count_kernel(SoftArgs a) {
    __shared__ int32_t s_cnt[kSoftMaxTileCount];
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const int nt = a.n_tiles;
    for (int t = tid; t < nt; t += 256) s_cnt[t] = 0;
    __syncthreads();
    const FaceRec* faces = a.faces + size_t(b) * a.total_faces;
    for (int32_t f = g * 256 + tid; f < a.total_faces; f += kSoftBinGroups * 256) {
        const FaceRec r = faces[f];
        if (r.orient == 0.0f) continue;
        int tx0, tx1, ty0, ty1;
        if (!face_tiles(r, tx0, tx1, ty0, ty1)) {
            a.big[size_t(b) * a.total_faces + atomicAdd(&a.big_n[b], 1)] = f;
            continue;
        }
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) atomicAdd(&s_cnt[ty * a.tiles_x + tx], 1);
    }
    __syncthreads();
    int32_t* first = a.tile_cnt + (size_t(b) * kSoftBinGroups + g) * nt;
    int32_t* tot = a.tile_tot + size_t(b) * nt;
    for (int t = tid; t < nt; t += 256)
        if (s_cnt[t] > 0) first[t] = atomicAdd(&tot[t], s_cnt[t]);
}

__global__ __launch_bounds__(256) void soft_bin_fill_kernel(SoftArgs a) {
    __shared__ int32_t s_cur[kSoftMaxTileCount];
    const int g = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const int nt = a.n_tiles;
    // tiles this workgroup did not count hold stale first slots; they are not touched below
    const int32_t* first = a.tile_cnt + (size_t(b) * kSoftBinGroups + g) * nt;
    const int32_t* off = a.tile_off + size_t(b) * (nt + 1);
    for (int t = tid; t < nt; t += 256) s_cur[t] = off[t] + first[t];
    __syncthreads();
    const FaceRec* faces = a.faces + size_t(b) * a.total_faces;
    int32_t* lists = a.lists + size_t(b) * a.total_faces * kSoftMaxTiles;
    for (int32_t f = g * 256 + tid; f < a.total_faces; f += kSoftBinGroups * 256) {
        const FaceRec r = faces[f];
        if (r.orient == 0.0f) continue;
        int tx0, tx1, ty0, ty1;
        if (!face_tiles(r, tx0, tx1, ty0, ty1)) continue;
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) lists[atomicAdd(&s_cur[ty * a.tiles_x + tx], 1)] = f;
    }
}

__device__ __forceinline__ int32_t fwd_items(int32_t n, int32_t chunk) { return n <= chunk ? 1 : (n + chunk - 1) / chunk; }

// Plan of the forward pass, one workgroup per candidate: the list offsets of
// the tiles (from the totals of the multi-workgroup binning when from_totals,
// else already written by the single-workgroup binning) and the work items:
// a tile whose list is longer than fwd_chunk faces is split into items of
// fwd_chunk faces, whose sums meet in facc (cleared here) and are
// finished by the last item to arrive (done, cleared here).
__global__ __launch_bounds__(kSoftBinThreads) void soft_plan_kernel(SoftArgs a, int from_totals) {
    __shared__ int32_t s_c[kSoftBinThreads], s_k[kSoftBinThreads];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int nt = a.n_tiles;
    int32_t* off = a.tile_off + size_t(b) * (nt + 1);
    const int32_t* tot = from_totals ? a.tile_tot + size_t(b) * nt : nullptr;
    const int per = (nt + kSoftBinThreads - 1) / kSoftBinThreads;
    const int c0 = min(tid * per, nt), c1 = min(c0 + per, nt);
    int32_t sc = 0, sk = 0;
    for (int t = c0; t < c1; t++) {
        const int32_t n = from_totals ? tot[t] : off[t + 1] - off[t];
        sc += n;
        sk += fwd_items(n, a.fwd_chunk);
    }
    s_c[tid] = sc;
    s_k[tid] = sk;
    __syncthreads();
    for (int o = 1; o < kSoftBinThreads; o <<= 1) {
        const int32_t vc = tid >= o ? s_c[tid - o] : 0, vk = tid >= o ? s_k[tid - o] : 0;
        __syncthreads();
        s_c[tid] += vc;
        s_k[tid] += vk;
        __syncthreads();
    }
    int32_t rc = s_c[tid] - sc, rk = s_k[tid] - sk;
    int2* items = a.chunks + size_t(b) * a.chunk_cap;
    const int lane = tid & 63;
    for (int i = 0; i < per; i++) {              // the same trip count on every lane
        const int t = c0 + i;
        const bool valid = t < c1;
        int32_t k_n = 0;
        if (valid) {
            const int32_t n = from_totals ? tot[t] : off[t + 1] - off[t];
            if (from_totals) off[t] = rc;
            rc += n;
            k_n = fwd_items(n, a.fwd_chunk);
            for (int32_t k = 0; k < k_n; k++) items[rk + k] = make_int2(t, k);
            rk += k_n;
            if (k_n > 1) a.done[size_t(b) * nt + t] = 0;
        }
        // the sums of split tiles, cleared by the whole wave one tile at a time
        // (one contiguous 512-byte store per tile)
        uint64_t split = __ballot(k_n > 1);
        while (split != 0ull) {
            const int src = __builtin_ctzll(split);
            split &= split - 1;
            const int ts = __shfl(t, src);
            a.facc[(size_t(b) * nt + ts) * 64 + lane] = 0;
        }
    }
    if (tid == kSoftBinThreads - 1) {
        if (from_totals) off[nt] = s_c[tid];
        a.chunk_n[b] = s_k[tid];
    }
}

// log(1 - prob) of one (pixel, face) pair in fixed point; 0 outside the band.
__device__ __forceinline__ long long pair_log_fixed(const FaceRec& r, int px, int py, float inv_sigma) {
    if (px < r.x0 || px > r.x1 || py < r.y0 || py > r.y1) return 0;
    const EdgeHit h = face_distance(r, px + 0.5f, py + 0.5f);
    const float x = h.d * inv_sigma;
    if (!(x >= -kBand)) return 0;
    const float term = softplus_f(-kBand) - softplus_f(x);
    return llrint(double(term) * kFixScale);
}

// One wave per work item (tile, k) of the candidate, looping when the grid
// is smaller than the item count; lane = pixel of the 8x8 tile, the wave adds
// the fixed-point terms of faces k * fwd_chunk ... of the tile list (item 0
// also of the big faces).  A tile of one item is finished at once; the items
// of a longer list add their sums into facc, and the last to arrive finishes
// the tile.  All sums are integers: the same bits in any order.
__device__ __forceinline__ void fwd_finish(const SoftArgs& a, const uint64_t* __restrict__ target,
                                           float* __restrict__ S_out, int b, int t, int lane, long long acc) {
    const int tx = t % a.tiles_x, ty = t / a.tiles_x;
    const int px = tx * kSoftTile + (lane & 7), py = ty * kSoftTile + (lane >> 3);
    const int W = a.cam.width, H = a.cam.height;
    const bool inimg = px < W && py < H;
    const double lsum = double(acc) / kFixScale;         // log(1 - S)
    const double one_minus_S = exp(lsum);
    const double S = -expm1(lsum);
    double m = 0.0;
    if (inimg) {
        const int bx = (W + 7) / 8;
        m = double((target[(py >> 3) * bx + (px >> 3)] >> ((py & 7) * 8 + (px & 7))) & 1ull);
    }
    double l = inimg ? (S - m) * (S - m) : 0.0;
    if (inimg) {
        a.G[size_t(b) * W * H + size_t(py) * W + px] = float(2.0 * (S - m) * one_minus_S * double(a.inv_sigma));
        if (S_out) S_out[size_t(b) * W * H + size_t(py) * W + px] = float(S);
    }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
    if (lane == 0) a.tloss[size_t(b) * a.n_tiles + t] = l;
}

// The read-only inputs come as separate restrict arguments: the kernel's own
// stores then provably leave them alone, and their wave-uniform loads stay
// scalar (face records in SGPRs) across the item loop.  The register bound
// (8 waves per SIMD) keeps the constants of fwd_finish's FP64 exp / expm1
// from being hoisted out of the loop into vector registers.
__global__ __launch_bounds__(64, 8) void soft_fwd_kernel(SoftArgs a, const FaceRec* __restrict__ faces_all,
                                                     const int32_t* __restrict__ lists_all,
                                                     const int32_t* __restrict__ off_all,
                                                     const int2* __restrict__ items_all,
                                                     const int32_t* __restrict__ big_all,
                                                     const uint64_t* __restrict__ target, float* __restrict__ S_out) {
    const int b = blockIdx.y;
    const int lane = threadIdx.x;
    const FaceRec* __restrict__ faces = faces_all + size_t(b) * a.total_faces;
    const int32_t* __restrict__ off = off_all + size_t(b) * (a.n_tiles + 1);
    const int32_t* __restrict__ lists = lists_all + size_t(b) * a.total_faces * kSoftMaxTiles;
    const int2* __restrict__ items = items_all + size_t(b) * a.chunk_cap;
    const int32_t n_items = a.chunk_n[b];
    const int32_t nb = a.big_n[b];
    const int32_t* __restrict__ big = big_all + size_t(b) * a.total_faces;
    for (int32_t c = blockIdx.x; c < n_items; c += gridDim.x) {
        const int2 it = items[c];
        const int t = it.x, k = it.y;
        const int tx = t % a.tiles_x, ty = t / a.tiles_x;
        const int px = tx * kSoftTile + (lane & 7), py = ty * kSoftTile + (lane >> 3);
        const int32_t e0 = off[t], e1 = off[t + 1];
        const int32_t k_n = fwd_items(e1 - e0, a.fwd_chunk);
        const int32_t lo = e0 + k * a.fwd_chunk, hi = min(lo + a.fwd_chunk, e1);
        long long acc = 0;
        for (int32_t e = lo; e < hi; e++) acc += pair_log_fixed(faces[lists[e]], px, py, a.inv_sigma);
        if (k == 0) {
            const int x_lo = tx * kSoftTile, y_lo = ty * kSoftTile;
            for (int32_t e = 0; e < nb; e++) {
                const FaceRec r = faces[big[e]];
                if (r.x1 < x_lo || r.x0 >= x_lo + kSoftTile || r.y1 < y_lo || r.y0 >= y_lo + kSoftTile) continue;
                acc += pair_log_fixed(r, px, py, a.inv_sigma);
            }
        }
        bool finish = true;
        if (k_n > 1) {
            long long* tacc = a.facc + (size_t(b) * a.n_tiles + t) * 64;
            atomicAdd(reinterpret_cast<unsigned long long*>(tacc + lane), static_cast<unsigned long long>(acc));
            __threadfence();
            int last = 0;
            if (lane == 0) last = atomicAdd(&a.done[size_t(b) * a.n_tiles + t], 1) == k_n - 1;
            finish = __shfl(last, 0) != 0;
            if (finish) {
                __threadfence();
                acc = static_cast<long long>(__hip_atomic_load(reinterpret_cast<unsigned long long*>(tacc + lane),
                                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
        }
        if (finish) fwd_finish(a, target, S_out, b, t, lane, acc);
    }
}

__global__ __launch_bounds__(256) void soft_loss_kernel(SoftArgs a, double* __restrict__ loss) {
    __shared__ double s[256];
    const int b = blockIdx.x, tid = threadIdx.x;
    const double* tl = a.tloss + size_t(b) * a.n_tiles;
    double acc = 0.0;
    for (int t = tid; t < a.n_tiles; t += 256) acc += tl[t];
    s[tid] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s[tid] += s[tid + o];
        __syncthreads();
    }
    if (tid == 0) loss[b] = s[0];
}

// ---------------------------------------------------------------- backward kernels

// One lane per face: dL/d(corners) over the pixels of its band, then through
// the pinhole projection into dL/dM_l; per-workgroup sums in a fixed order.
__global__ __launch_bounds__(kSoftFaceBlock) void soft_bwd_face_kernel(SoftArgs a) {
    __shared__ float s_acc[kSoftGrad][kSoftFaceBlock + 1];
    const int b = blockIdx.y;
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    // kSoftFaceLanes lanes per face: lane j of a group walks the band rows y0 + j, y0 + j + kSoftFaceLanes, ...
    const int grp = tid / kSoftFaceLanes, j = tid % kSoftFaceLanes;
    const int arm = (a.ms.n_meshes > 1 && blk >= a.block_offset[1]) ? 1 : 0;
    const MeshK m = arm == 0 ? a.ms.m[0] : a.ms.m[1];
    const int32_t lf = (blk - (arm == 0 ? 0 : a.block_offset[1])) * kSoftFacesPerBlock + grp;
    const int32_t gf = (arm == 0 ? a.face_offset[0] : a.face_offset[1]) + lf;
    float acc[kSoftGrad];
#pragma unroll
    for (int e = 0; e < kSoftGrad; e++) acc[e] = 0.0f;
    const bool has = lf < m.n_triangles;
    FaceRec r;
    if (has) r = a.faces[size_t(b) * a.total_faces + gf];
    const bool live = has && r.orient != 0.0f;
    float g0u = 0.0f, g0v = 0.0f, g1u = 0.0f, g1v = 0.0f, g2u = 0.0f, g2v = 0.0f;
    if (live) {
        const int W = a.cam.width;
        const float* Gm = a.G + size_t(b) * W * a.cam.height;
        for (int py = r.y0 + j; py <= r.y1; py += kSoftFaceLanes) {
            for (int px = r.x0; px <= r.x1; px++) {
                const float G = Gm[size_t(py) * W + px];
                if (G == 0.0f) continue;
                const EdgeHit h = face_distance(r, px + 0.5f, py + 0.5f);
                const float x = h.d * a.inv_sigma;
                if (!(x >= -kBand)) continue;
                const float sg = 1.0f / (1.0f + expf(-x));
                // dL/dd = G sig(x); dd/d(corner a) = -sg n (1 - t), dd/d(corner b) = -sg n t
                const float w = -G * sg * h.sg;
                const float wa = w * (1.0f - h.t), wb = w * h.t;
                const int ia = h.ia, ib = ia == 2 ? 0 : ia + 1;
                const float ca0 = ia == 0 ? wa : (ib == 0 ? wb : 0.0f);
                const float ca1 = ia == 1 ? wa : (ib == 1 ? wb : 0.0f);
                const float ca2 = ia == 2 ? wa : (ib == 2 ? wb : 0.0f);
                g0u += ca0 * h.nx;
                g0v += ca0 * h.ny;
                g1u += ca1 * h.nx;
                g1v += ca1 * h.ny;
                g2u += ca2 * h.nx;
                g2v += ca2 * h.ny;
            }
        }
    }
    // the face's corner gradients: butterfly over its lanes (fixed order; lane 0's sum is used)
#pragma unroll
    for (int o = 1; o < kSoftFaceLanes; o <<= 1) {
        g0u += __shfl_xor(g0u, o);
        g0v += __shfl_xor(g0v, o);
        g1u += __shfl_xor(g1u, o);
        g1v += __shfl_xor(g1v, o);
        g2u += __shfl_xor(g2u, o);
        g2v += __shfl_xor(g2v, o);
    }
    if (live && j == 0) {
        const float4* V = a.verts + size_t(b) * a.ms.total_vertices + m.vertex_offset;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const float gu = c == 0 ? g0u : (c == 1 ? g1u : g2u);
            const float gv = c == 0 ? g0v : (c == 1 ? g1v : g2v);
            const int32_t vi = m.triangles[3 * lf + c];
            const float4 p = V[vi];
            const float iz = 1.0f / p.z;
            // u = fx X / Z + cx: dL/dX = gu fx / Z, dL/dY = gv fy / Z,
            // dL/dZ = -(gu (u - cx) + gv (v - cy)) / Z
            const float gX = gu * a.cam.fx * iz, gY = gv * a.cam.fy * iz;
            const float gZ = -(gu * (p.x - a.cam.cx) + gv * (p.y - a.cam.cy)) * iz;
            const float h4[4] = {m.vertices[3 * vi], m.vertices[3 * vi + 1], m.vertices[3 * vi + 2], 1.0f};
            const int l = m.vertex_link[vi];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const float e0 = gX * h4[k], e1 = gY * h4[k], e2 = gZ * h4[k];
#pragma unroll
                for (int ll = 0; ll < 4; ll++) {
                    if (l == ll) {
                        acc[ll * 12 + k] += e0;
                        acc[ll * 12 + 4 + k] += e1;
                        acc[ll * 12 + 8 + k] += e2;
                    }
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < kSoftGrad; e++) s_acc[e][tid] = acc[e];
    __syncthreads();
    // fixed-order tree over the lanes of each entry
    for (int o = kSoftFaceBlock / 2; o > 0; o >>= 1) {
        for (int idx = tid; idx < kSoftGrad * o; idx += kSoftFaceBlock) {
            const int e = idx / o, jj = idx % o;
            s_acc[e][jj] += s_acc[e][jj + o];
        }
        __syncthreads();
    }
    if (tid < kSoftGrad) a.part[(size_t(b) * a.n_blocks + blk) * kSoftGrad + tid] = s_acc[tid][0];
}

struct ChainD {
    double d, lb[3], ub[3];
};

struct ParamArgs {
    ChainD ch[kMaxArms];
    const float* X;          // [batch][9 n_arms]
    const double* grad_loss; // nullable [batch]
    float* grad_X;           // [batch][9 n_arms]
};

// 3x3 products and the elementary rotations with their derivatives (FP64)
__device__ inline void mm3(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
__device__ inline void rot_and_deriv(int axis, double a, double* R, double* D) {
    const double c = cos(a), s = sin(a);
    for (int i = 0; i < 9; i++) R[i] = D[i] = 0.0;
    if (axis == 0) {          // x
        R[0] = 1; R[4] = c; R[5] = -s; R[7] = s; R[8] = c;
        D[4] = -s; D[5] = -c; D[7] = c; D[8] = -s;
    } else if (axis == 1) {   // y
        R[0] = c; R[2] = s; R[4] = 1; R[6] = -s; R[8] = c;
        D[0] = -s; D[2] = c; D[6] = -c; D[8] = -s;
    } else {                  // z
        R[0] = c; R[1] = -s; R[3] = s; R[4] = c; R[8] = 1;
        D[0] = -s; D[1] = -c; D[3] = c; D[4] = -s;
    }
}

// <G, [A | a]> with G a 3x4 gradient, A 3x3, a 3-vector
__device__ inline double dot34(const double* G, const double* A, const double* a) {
    double s = 0.0;
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) s += G[4 * r + c] * A[3 * r + c];
        s += G[4 * r + 3] * a[r];
    }
    return s;
}

// Sum of the workgroup partials (fixed order) and the Jacobian of
// M_l = T_r^c(alpha, beta, gamma, x, y, z) T_l(q(qhat)):
// T_r^c = [Ry(gamma) Rx(alpha) Rz(beta) | (x, y, z)], T_0 = I, T_1 = Rx(q1),
// T_2,3 = [Rx(q1) Ry(q2 +- q3/2) | Rx(q1) (0, 0, d)], q = lb + (ub - lb)/2 (1 - cos(pi (qhat - lb)/(ub - lb))).
constexpr int kParamThreads = 128;

// Sums of the per-workgroup partials of dL/dM_l of one candidate in a fixed
// order: workgroup g takes the g-th of kSoftReduceGroups contiguous slices of
// each arm's rows; in it, wave w adds rows w, w + 4, ... with lane e on entry e
// (coalesced 48-float rows), then the waves' sums are added in order.
__global__ __launch_bounds__(256) void soft_reduce_kernel(SoftArgs a) {
    __shared__ double s_w[4][kMaxArms * kSoftGrad];
    const int g = blockIdx.x, b = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n_arms = a.ms.n_meshes;
    for (int arm = 0; arm < n_arms; arm++) {
        const int r0 = arm == 0 ? 0 : a.block_offset[1];
        const int r1 = (arm == 0 && n_arms > 1) ? a.block_offset[1] : a.n_blocks;
        const int k0 = r0 + int((long long)(r1 - r0) * g / kSoftReduceGroups);
        const int k1 = r0 + int((long long)(r1 - r0) * (g + 1) / kSoftReduceGroups);
        double s = 0.0;
        if (lane < kSoftGrad) {
            const float* row = a.part + size_t(b) * a.n_blocks * kSoftGrad + lane;
#pragma unroll 4
            for (int k = k0 + w; k < k1; k += 4) s += double(row[size_t(k) * kSoftGrad]);
            s_w[w][arm * kSoftGrad + lane] = s;
        }
    }
    __syncthreads();
    if (threadIdx.x < n_arms * kSoftGrad)
        a.gsum[(size_t(b) * kSoftReduceGroups + g) * kMaxArms * kSoftGrad + threadIdx.x] =
            ((s_w[0][threadIdx.x] + s_w[1][threadIdx.x]) + s_w[2][threadIdx.x]) + s_w[3][threadIdx.x];
}

// Jacobian of the link transforms applied to the summed dL/dM_l.
__global__ __launch_bounds__(kParamThreads) void soft_param_kernel(SoftArgs a, ParamArgs p) {
    __shared__ double s_g[kMaxArms][kSoftGrad];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int n_arms = a.ms.n_meshes;
    if (tid < n_arms * kSoftGrad) {
        double v = 0.0;
        for (int g = 0; g < kSoftReduceGroups; g++) v += a.gsum[(size_t(b) * kSoftReduceGroups + g) * kMaxArms * kSoftGrad + tid];
        s_g[tid / kSoftGrad][tid % kSoftGrad] = v;
    }
    __syncthreads();
    if (tid >= n_arms) return;
    const int arm = tid;
    const ChainD ch = arm == 0 ? p.ch[0] : p.ch[1];
    const float* th = p.X + (size_t(b) * n_arms + arm) * 9;
    double Rx_[9], dRx[9], Ry_[9], dRy[9], Rz_[9], dRz[9], t1[9], R[9], dR[3][9];
    rot_and_deriv(0, double(th[0]), Rx_, dRx);
    rot_and_deriv(2, double(th[1]), Rz_, dRz);
    rot_and_deriv(1, double(th[2]), Ry_, dRy);
    mm3(Ry_, Rx_, t1);
    mm3(t1, Rz_, R);
    mm3(Ry_, dRx, t1);
    mm3(t1, Rz_, dR[0]);          // d/d alpha
    mm3(Ry_, Rx_, t1);
    mm3(t1, dRz, dR[1]);          // d/d beta
    mm3(dRy, Rx_, t1);
    mm3(t1, Rz_, dR[2]);          // d/d gamma
    double q[3], dq[3];
    for (int j = 0; j < 3; j++) {
        const double lb = ch.lb[j], ub = ch.ub[j];
        const double ang = 3.14159265358979323846 * (double(th[6 + j]) - lb) / (ub - lb);
        q[j] = lb + (ub - lb) * 0.5 * (1.0 - cos(ang));
        dq[j] = 1.57079632679489661923 * sin(ang);
    }
    // link rotations / translations and their derivatives in q1 and in the jaw angle phi
    double Lr[4][9], Lt[4][3], dLr_q1[4][9], dLt_q1[4][3], dLr_phi[4][9];
    double Q1[9], dQ1[9];
    rot_and_deriv(0, q[0], Q1, dQ1);
    for (int l = 0; l < 4; l++)
        for (int i = 0; i < 9; i++) Lr[l][i] = dLr_q1[l][i] = dLr_phi[l][i] = 0.0;
    for (int l = 0; l < 4; l++)
        for (int i = 0; i < 3; i++) Lt[l][i] = dLt_q1[l][i] = 0.0;
    Lr[0][0] = Lr[0][4] = Lr[0][8] = 1.0;
    for (int i = 0; i < 9; i++) {
        Lr[1][i] = Q1[i];
        dLr_q1[1][i] = dQ1[i];
    }
    for (int side = 0; side < 2; side++) {
        const double phi = side == 0 ? q[1] + 0.5 * q[2] : q[1] - 0.5 * q[2];
        double P[9], dP[9];
        rot_and_deriv(1, phi, P, dP);
        mm3(Q1, P, Lr[2 + side]);
        mm3(dQ1, P, dLr_q1[2 + side]);
        mm3(Q1, dP, dLr_phi[2 + side]);
        for (int i = 0; i < 3; i++) {
            Lt[2 + side][i] = Q1[3 * i + 2] * ch.d;
            dLt_q1[2 + side][i] = dQ1[3 * i + 2] * ch.d;
        }
    }
    double g[9];
    for (int k = 0; k < 9; k++) g[k] = 0.0;
    for (int l = 0; l < 4; l++) {
        const double* Gl = &s_g[arm][12 * l];
        double A[9], at[3];
        for (int k = 0; k < 3; k++) {            // rotation parameters: [dR L_rot | dR L_t]
            mm3(dR[k], Lr[l], A);
            for (int i = 0; i < 3; i++) at[i] = dR[k][3 * i] * Lt[l][0] + dR[k][3 * i + 1] * Lt[l][1] + dR[k][3 * i + 2] * Lt[l][2];
            g[k] += dot34(Gl, A, at);
        }
        for (int k = 0; k < 3; k++) g[3 + k] += Gl[4 * k + 3];   // translation: [0 | e_k]
        // joints: [R dL_rot | R dL_t] dq/dqhat
        mm3(R, dLr_q1[l], A);
        for (int i = 0; i < 3; i++) at[i] = R[3 * i] * dLt_q1[l][0] + R[3 * i + 1] * dLt_q1[l][1] + R[3 * i + 2] * dLt_q1[l][2];
        g[6] += dot34(Gl, A, at) * dq[0];
        if (l >= 2) {
            const double z3[3] = {0.0, 0.0, 0.0};
            mm3(R, dLr_phi[l], A);
            const double gphi = dot34(Gl, A, z3);
            g[7] += gphi * dq[1];
            g[8] += (l == 2 ? 0.5 : -0.5) * gphi * dq[2];
        }
    }
    const double scale = p.grad_loss ? p.grad_loss[b] : 1.0;
    for (int k = 0; k < 9; k++) p.grad_X[(size_t(b) * n_arms + arm) * 9 + k] = float(g[k] * scale);
}

// Shapes and layout (no workspace needed).
tk_status make_soft_shape(int32_t batch, const tk_mesh* meshes, int32_t n_meshes, const tk_camera* cam,
                          float sigma, SoftArgs* a, SoftLayout* L) {
    TK_REQUIRE(batch >= 0 && batch <= 65535, "batch = %d outside 0..65535", batch);
    TK_REQUIRE(std::isfinite(sigma) && sigma > 0.0f && sigma <= 64.0f, "sigma must be in (0, 64] pixels");
    std::memset(a, 0, sizeof *a);
    if (tk_status st = validate_meshes(meshes, n_meshes, &a->ms)) return st;
    if (tk_status st = validate_camera(cam)) return st;
    a->cam = make_cam(*cam);
    int32_t fpa[kMaxArms] = {0, 0};
    int64_t total = 0;
    for (int i = 0; i < n_meshes; i++) {
        a->face_offset[i] = int32_t(total);
        fpa[i] = meshes[i].n_triangles;
        total += meshes[i].n_triangles;
    }
    TK_REQUIRE(total <= (1 << 24), "more than 16M faces");
    a->total_faces = int32_t(total);
    a->batch = batch;
    a->sigma = sigma;
    a->inv_sigma = 1.0f / sigma;
    *L = soft_layout(batch, a->ms, a->total_faces, cam->width, cam->height, fpa);
    if (L->n_tiles > kSoftMaxTileCount)
        return fail(TK_ERR_UNSUPPORTED, "image of %d 8x8 tiles exceeds the soft path's %d (1024x1024 fits)",
                    L->n_tiles, kSoftMaxTileCount);
    a->tiles_x = L->tiles_x;
    a->tiles_y = L->tiles_y;
    a->n_tiles = L->n_tiles;
    a->n_blocks = L->n_blocks;
    a->chunk_cap = L->chunk_cap;
    a->fwd_chunk = L->fwd_chunk;
    a->block_offset[0] = 0;
    a->block_offset[1] = (fpa[0] + kSoftFacesPerBlock - 1) / kSoftFacesPerBlock;
    return TK_OK;
}

// Shapes, layout and the workspace pointers.
tk_status make_soft_args(int32_t batch, const tk_mesh* meshes, int32_t n_meshes, const tk_camera* cam, float sigma,
                         void* d_ws, size_t ws_bytes, SoftArgs* a, SoftLayout* L) {
    if (tk_status st = make_soft_shape(batch, meshes, n_meshes, cam, sigma, a, L)) return st;
    if (batch == 0) return TK_OK;
    TK_REQUIRE(d_ws != nullptr, "workspace is NULL");
    if (ws_bytes < L->total)
        return fail(TK_ERR_WORKSPACE_TOO_SMALL, "soft workspace of %zu bytes, %zu needed", ws_bytes, L->total);
    TK_REQUIRE((reinterpret_cast<uintptr_t>(d_ws) & 255) == 0, "workspace must be 256-byte aligned");
    char* w = static_cast<char*>(d_ws);
    a->verts = reinterpret_cast<float4*>(w + L->verts);
    a->faces = reinterpret_cast<FaceRec*>(w + L->faces);
    a->tile_off = reinterpret_cast<int32_t*>(w + L->tile_off);
    a->tile_cnt = reinterpret_cast<int32_t*>(w + L->tile_cnt);
    a->tile_tot = batch < kSoftWideBin ? reinterpret_cast<int32_t*>(w + L->tile_tot) : nullptr;
    a->chunks = reinterpret_cast<int2*>(w + L->chunks);
    a->chunk_n = reinterpret_cast<int32_t*>(w + L->chunk_n);
    a->facc = reinterpret_cast<long long*>(w + L->facc);
    a->done = reinterpret_cast<int32_t*>(w + L->done);
    a->lists = reinterpret_cast<int32_t*>(w + L->lists);
    a->big = reinterpret_cast<int32_t*>(w + L->big);
    a->big_n = reinterpret_cast<int32_t*>(w + L->big_n);
    a->G = reinterpret_cast<float*>(w + L->G);
    a->tloss = reinterpret_cast<double*>(w + L->tloss);
    a->part = reinterpret_cast<float*>(w + L->part);
    a->gsum = reinterpret_cast<double*>(w + L->gsum);
    return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

size_t tk_soft_workspace_bytes(int32_t batch, const tk_mesh* meshes, int32_t n_meshes, const tk_camera* cam) {
    clear_error();
    SoftArgs a;
    SoftLayout L;
    if (make_soft_shape(batch, meshes, n_meshes, cam, 1.0f, &a, &L) != TK_OK) return 0;
    return L.total;
}

tk_status tk_soft_forward(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                          const tk_camera* cam, float sigma, const uint64_t* d_target, float* d_S, double* d_loss,
                          void* d_ws, size_t ws_bytes, tk_stream s) {
    clear_error();
    SoftArgs a;
    SoftLayout L;
    if (tk_status st = make_soft_args(batch, meshes, n_meshes, cam, sigma, d_ws, ws_bytes, &a, &L)) return st;
    if (batch == 0) return TK_OK;
    TK_REQUIRE(d_link_xf && d_target && d_loss, "link_xf / target / loss is NULL");
    hipStream_t st = reinterpret_cast<hipStream_t>(s);
    hipLaunchKernelGGL(soft_vert_kernel, dim3((a.ms.total_vertices + 255) / 256, batch), dim3(256), 0, st, d_link_xf,
                       a);
    const int face_blocks = (a.total_faces + 255) / 256;
    hipLaunchKernelGGL(soft_face_kernel, dim3(face_blocks > 0 ? face_blocks : 1, batch), dim3(256), 0, st, a);
    if (batch >= kSoftWideBin) {
        hipLaunchKernelGGL(soft_bin_kernel, dim3(batch), dim3(kSoftBinThreads), 0, st, a);
        hipLaunchKernelGGL(soft_plan_kernel, dim3(batch), dim3(kSoftBinThreads), 0, st, a, 0);
    } else {
        hipLaunchKernelGGL(soft_bin_count_kernel, dim3(kSoftBinGroups, batch), dim3(256), 0, st, a);
        hipLaunchKernelGGL(soft_plan_kernel, dim3(batch), dim3(kSoftBinThreads), 0, st, a, 1);
        hipLaunchKernelGGL(soft_bin_fill_kernel, dim3(kSoftBinGroups, batch), dim3(256), 0, st, a);
    }
    // a wave per work item (an item per tile, and the extra items of split
    // tiles), looping when a candidate has more items than the grid
    const int fwd_groups = std::min(a.chunk_cap, 2 * a.n_tiles);
    hipLaunchKernelGGL(soft_fwd_kernel, dim3(fwd_groups, batch), dim3(64), 0, st, a, a.faces, a.lists, a.tile_off,
                       a.chunks, a.big, d_target, d_S);
    hipLaunchKernelGGL(soft_loss_kernel, dim3(batch), dim3(256), 0, st, a, d_loss);
    return check_launch("tk_soft_forward");
}

tk_status tk_soft_backward(const float* d_X, int32_t batch, const tk_chain* chains, const tk_mesh* meshes,
                           int32_t n_arms, const tk_camera* cam, float sigma, const double* d_grad_loss,
                           float* d_grad_X, void* d_ws, size_t ws_bytes, tk_stream s) {
    clear_error();
    SoftArgs a;
    SoftLayout L;
    if (tk_status st = make_soft_args(batch, meshes, n_arms, cam, sigma, d_ws, ws_bytes, &a, &L)) return st;
    TK_REQUIRE(chains != nullptr, "chains is NULL");
    ParamArgs p;
    std::memset(&p, 0, sizeof p);
    for (int i = 0; i < n_arms; i++) {
        p.ch[i].d = chains[i].d_pitch_yaw;
        for (int j = 0; j < 3; j++) {
            TK_REQUIRE(chains[i].q_ub[j] > chains[i].q_lb[j], "chain %d: joint %d has q_ub <= q_lb", i, j);
            p.ch[i].lb[j] = chains[i].q_lb[j];
            p.ch[i].ub[j] = chains[i].q_ub[j];
        }
    }
    if (batch == 0) return TK_OK;
    TK_REQUIRE(d_X && d_grad_X, "X / grad_X is NULL");
    p.X = d_X;
    p.grad_loss = d_grad_loss;
    p.grad_X = d_grad_X;
    hipStream_t st = reinterpret_cast<hipStream_t>(s);
    if (a.n_blocks > 0)
        hipLaunchKernelGGL(soft_bwd_face_kernel, dim3(a.n_blocks, batch), dim3(kSoftFaceBlock), 0, st, a);
    hipLaunchKernelGGL(soft_reduce_kernel, dim3(kSoftReduceGroups, batch), dim3(256), 0, st, a);
    hipLaunchKernelGGL(soft_param_kernel, dim3(batch), dim3(kParamThreads), 0, st, a, p);
    return check_launch("tk_soft_backward");
}

}  // extern "C"
