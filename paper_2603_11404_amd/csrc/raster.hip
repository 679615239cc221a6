// Binary silhouette rasterisation and mask counts on gfx950 (wave64).
//
// Renderer S = R(K(Pi(T_r^c T_m^r(q) v_m))) of paper Sec. III-A.2 with
// S in {0,1}^{H x W}; counts |S| and |S and M_ref| feed the render loss
// (Eq. render_loss) and the mask error 1 - IoU (Sec. IV).
//
// Design (one workgroup per candidate, whole image mask in LDS):
//   1. each lane takes one triangle: gathers its three vertices, applies the
//      link transform of the candidate (FP32, no contraction), projects with
//      the pinhole camera and snaps to Q8 fixed point; culls triangles with a
//      vertex before the near plane, zero area or an empty pixel box;
//      orients the triangle and builds three exact integer edge functions
//      E(p) = dx*(p.y - y0) - dy*(p.x - x0) with the top-left bias; stores a
//      64-byte record in the wave's LDS staging slot;
//   2. the wave walks its valid triangles one by one; for every 8x8 pixel
//      block of the triangle's box, each lane tests its pixel centre with the
//      three edge functions (32-bit modular arithmetic, exact because the box
//      bound keeps |E| < 2^31; a 64-bit path serves larger triangles) and
//      the 64-lane ballot is the block's coverage word, ORed into the LDS
//      mask with one ds_or_b64;
//   3. after a barrier the mask is written out and/or reduced against the
//      target with popcounts.
#include <cstring>
#include <mutex>

#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------- vertex transform

// FP32 transform p = M [v; 1], pinhole projection and Q8 snap (round half to
// even).  Returns false when the vertex is culled (Z < z_near or NaN).
__device__ __forceinline__ bool project_snap(const float* __restrict__ M, float vx, float vy, float vz,
                                             const CamK& cam, int32_t& X, int32_t& Y) {
#pragma clang fp contract(off)
    const float px = ((M[0] * vx + M[1] * vy) + M[2] * vz) + M[3];
    const float py = ((M[4] * vx + M[5] * vy) + M[6] * vz) + M[7];
    const float pz = ((M[8] * vx + M[9] * vy) + M[10] * vz) + M[11];
    float u = cam.fx * (px / pz) + cam.cx;
    float v = cam.fy * (py / pz) + cam.cy;
    const bool ok = (pz >= cam.z_near) && (u == u) && (v == v);
    u = fminf(fmaxf(u, -32768.0f), 32768.0f);
    v = fminf(fmaxf(v, -32768.0f), 32768.0f);
    X = ok ? int32_t(rintf(u * 256.0f)) : INT32_MIN;
    Y = ok ? int32_t(rintf(v * 256.0f)) : 0;
    return ok;
}

// ---------------------------------------------------------------- triangle setup

struct TriRec {            // 64 bytes
    int64_t e0[3];         // edge functions (with bias) at the centre of the first block's first pixel
    int32_t dx[3], dy[3];  // edge vectors in Q8 units
    int32_t bx0, by0;      // first block
    int32_t nbx, nby;      // blocks spanned; nby bit 16 = needs 64-bit evaluation
};
static_assert(sizeof(TriRec) == 64, "record size");

constexpr int32_t kHugeBit = 1 << 16;

// Builds the record of one triangle from its snapped vertices; false if culled.
__device__ __forceinline__ bool setup_triangle(int32_t x0, int32_t y0, int32_t x1, int32_t y1, int32_t x2,
                                               int32_t y2, const CamK& cam, TriRec& r) {
    if (x0 == INT32_MIN || x1 == INT32_MIN || x2 == INT32_MIN) return false;
    const int64_t area2 = int64_t(x1 - x0) * int64_t(y2 - y0) - int64_t(y1 - y0) * int64_t(x2 - x0);
    if (area2 == 0) return false;
    if (area2 < 0) {  // orient positively (swap b and c)
        int32_t t = x1; x1 = x2; x2 = t;
        t = y1; y1 = y2; y2 = t;
    }
    const int32_t xmin = min(x0, min(x1, x2)), xmax = max(x0, max(x1, x2));
    const int32_t ymin = min(y0, min(y1, y2)), ymax = max(y0, max(y1, y2));
    // pixel centres 256 p + 128 inside [min, max]
    int32_t px0 = (xmin - 128 + 255) >> 8, px1 = (xmax - 128) >> 8;
    int32_t py0 = (ymin - 128 + 255) >> 8, py1 = (ymax - 128) >> 8;
    px0 = max(px0, 0);
    py0 = max(py0, 0);
    px1 = min(px1, cam.width - 1);
    py1 = min(py1, cam.height - 1);
    if (px0 > px1 || py0 > py1) return false;
    r.bx0 = px0 >> 3;
    r.by0 = py0 >> 3;
    r.nbx = (px1 >> 3) - r.bx0 + 1;
    r.nby = (py1 >> 3) - r.by0 + 1;
    const int32_t vx[3] = {x0, x1, x2}, vy[3] = {y0, y1, y2};
    const int64_t ox = int64_t(256) * (8 * r.bx0) + 128, oy = int64_t(256) * (8 * r.by0) + 128;
    bool huge = false;
    for (int e = 0; e < 3; e++) {
        const int n = e == 2 ? 0 : e + 1;
        const int32_t dx = vx[n] - vx[e], dy = vy[n] - vy[e];
        const bool top_left = (dy < 0) || (dy == 0 && dx > 0);
        const int64_t E = int64_t(dx) * (oy - vy[e]) - int64_t(dy) * (ox - vx[e]) + (top_left ? 0 : -1);
        r.e0[e] = E;
        r.dx[e] = dx;
        r.dy[e] = dy;
        // largest |E| over every pixel centre of the spanned blocks
        const int64_t a = int64_t(256) * (dy < 0 ? -int64_t(dy) : int64_t(dy));
        const int64_t b = int64_t(256) * (dx < 0 ? -int64_t(dx) : int64_t(dx));
        const int64_t bound = (E < 0 ? -E : E) + a * (8 * r.nbx - 1) + b * (8 * r.nby - 1);
        huge |= bound >= (int64_t(1) << 31);
    }
    if (huge) r.nby |= kHugeBit;
    return true;
}

// ---------------------------------------------------------------- coverage of one triangle

__device__ __forceinline__ void cover_triangle(const TriRec& r, int lx, int ly, int lane,
                                               unsigned long long* __restrict__ s_mask, int words_x) {
    const int bx0 = __builtin_amdgcn_readfirstlane(r.bx0);
    const int by0 = __builtin_amdgcn_readfirstlane(r.by0);
    const int nbx = __builtin_amdgcn_readfirstlane(r.nbx);
    const int nby_raw = __builtin_amdgcn_readfirstlane(r.nby);
    const int nby = nby_raw & 0xffff;
    if (!(nby_raw & kHugeBit)) {
        // 32-bit modular evaluation: E(lane, block) = L + bx*8A + by*8B, exact since |E| < 2^31
        uint32_t L[3], SX[3], SY[3];
        for (int e = 0; e < 3; e++) {
            const uint32_t A = 0u - (uint32_t(r.dy[e]) << 8);  // per pixel step in x: -256 dy
            const uint32_t B = uint32_t(r.dx[e]) << 8;         // per pixel step in y: +256 dx
            L[e] = A * uint32_t(lx) + B * uint32_t(ly) + uint32_t(r.e0[e]);
            SX[e] = A * 8u;
            SY[e] = B * 8u;
        }
        for (int by = 0; by < nby; by++) {
            uint32_t E0 = L[0], E1 = L[1], E2 = L[2];
            for (int bx = 0; bx < nbx; bx++) {
                const bool in = int32_t(E0 | E1 | E2) >= 0;
                const unsigned long long m = __ballot(in);
                if (m != 0ull && lane == 0) atomicOr(&s_mask[(by0 + by) * words_x + bx0 + bx], m);
                E0 += SX[0];
                E1 += SX[1];
                E2 += SX[2];
            }
            L[0] += SY[0];
            L[1] += SY[1];
            L[2] += SY[2];
        }
    } else {
        // 64-bit evaluation for triangles whose edge functions exceed 32 bits
        for (int by = 0; by < nby; by++) {
            for (int bx = 0; bx < nbx; bx++) {
                const int64_t px = 8 * bx + lx, py = 8 * by + ly;   // pixel offset from the record origin
                bool in = true;
                for (int e = 0; e < 3; e++) {
                    const int64_t E = r.e0[e] - int64_t(256) * r.dy[e] * px + int64_t(256) * r.dx[e] * py;
                    in = in && (E >= 0);
                }
                const unsigned long long m = __ballot(in);
                if (m != 0ull && lane == 0) atomicOr(&s_mask[(by0 + by) * words_x + bx0 + bx], m);
            }
        }
    }
}

// ---------------------------------------------------------------- valid-pixel masks of edge words

__device__ __forceinline__ unsigned long long valid_bits(int wx, int wy, const CamK& cam) {
    unsigned long long m = ~0ull;
    const int rx = cam.width - 8 * wx;   // valid columns in this word (>= 1)
    if (rx < 8) m &= 0x0101010101010101ull * ((1ull << rx) - 1ull);
    const int ry = cam.height - 8 * wy;
    if (ry < 8) m &= (1ull << (8 * ry)) - 1ull;
    return m;
}

// ---------------------------------------------------------------- main kernel

struct RasterArgs {
    MeshSet meshes;
    CamK cam;
    const float* link_xf;        // [batch][n_meshes][4][12]
    const int32_t* snapped;      // [batch][total V][2]
    unsigned long long* masks;   // [batch][words]
    const unsigned long long* target;
    int32_t* counts;             // [batch][2]
    int32_t batch;
};

template <bool FROM_SNAPPED, bool WRITE_MASK, bool COUNTS, int NT>
__global__ __launch_bounds__(NT) void raster_kernel(RasterArgs a) {
    constexpr int NW = NT / kWave;
    extern __shared__ unsigned long long s_mask[];
    __shared__ TriRec s_rec[NW][kWave];
    __shared__ float s_M[kMaxArms * 48];
    __shared__ int32_t s_red[2][NW];

    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int lx = lane & 7, ly = lane >> 3;
    const CamK& cam = a.cam;
    const int words = cam.words_x * cam.words_y;

    for (int w = tid; w < words; w += NT) s_mask[w] = 0ull;
    if (!FROM_SNAPPED)
        for (int i = tid; i < a.meshes.n_meshes * 48; i += NT)
            s_M[i] = a.link_xf[size_t(b) * a.meshes.n_meshes * 48 + i];
    __syncthreads();

    for (int mi = 0; mi < a.meshes.n_meshes; mi++) {
        const MeshK& mesh = a.meshes.m[mi];
        const float* M = s_M + mi * 48;
        for (int base = wave * kWave; base < mesh.n_triangles; base += NT) {
            const int t = base + lane;
            bool valid = false;
            TriRec rec;
            if (t < mesh.n_triangles) {
                const int32_t i0 = mesh.triangles[3 * t], i1 = mesh.triangles[3 * t + 1],
                              i2 = mesh.triangles[3 * t + 2];
                int32_t X[3], Y[3];
                const int32_t idx[3] = {i0, i1, i2};
                for (int k = 0; k < 3; k++) {
                    if (FROM_SNAPPED) {
                        const int32_t* p =
                            a.snapped + (size_t(b) * a.meshes.total_vertices + mesh.vertex_offset + idx[k]) * 2;
                        X[k] = p[0];
                        Y[k] = p[1];
                    } else {
                        const float* v = mesh.vertices + size_t(idx[k]) * 3;
                        const int link = mesh.vertex_link[idx[k]];
                        project_snap(M + 12 * link, v[0], v[1], v[2], cam, X[k], Y[k]);
                    }
                }
                valid = setup_triangle(X[0], Y[0], X[1], Y[1], X[2], Y[2], cam, rec);
            }
            if (valid) s_rec[wave][lane] = rec;
            unsigned long long todo = __ballot(valid);
            // records written by other lanes of this wave must be visible before they are read
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            while (todo) {
                const int j = __builtin_ctzll(todo);
                todo &= todo - 1;
                const TriRec r = s_rec[wave][j];
                cover_triangle(r, lx, ly, lane, s_mask, cam.words_x);
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();

    int32_t cnt_s = 0, cnt_i = 0;
    for (int w = tid; w < words; w += NT) {
        const int wy = w / cam.words_x, wx = w - wy * cam.words_x;
        const unsigned long long v = s_mask[w] & valid_bits(wx, wy, cam);
        if (WRITE_MASK) a.masks[size_t(b) * words + w] = v;
        if (COUNTS) {
            cnt_s += __popcll(v);
            cnt_i += __popcll(v & a.target[w]);
        }
    }
    if (COUNTS) {
        for (int off = kWave / 2; off > 0; off >>= 1) {
            cnt_s += __shfl_xor(cnt_s, off);
            cnt_i += __shfl_xor(cnt_i, off);
        }
        if (lane == 0) {
            s_red[0][wave] = cnt_s;
            s_red[1][wave] = cnt_i;
        }
        __syncthreads();
        if (tid == 0) {
            int32_t ts = 0, ti = 0;
            for (int w = 0; w < NW; w++) {
                ts += s_red[0][w];
                ti += s_red[1][w];
            }
            a.counts[2 * b] = ts;
            a.counts[2 * b + 1] = ti;
        }
    }
}

constexpr int kRasterThreads = 512;

// ---------------------------------------------------------------- snapped vertices (debug / parity)

struct SnapArgs {
    MeshSet meshes;
    CamK cam;
    const float* link_xf;
    int32_t* snapped;
    int32_t batch;
};

__global__ __launch_bounds__(256) void snap_kernel(SnapArgs a) {
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int TV = a.meshes.total_vertices;
    if (idx >= int64_t(a.batch) * TV) return;
    const int b = int(idx / TV), gv = int(idx % TV);
    int mi = 0;
    while (mi + 1 < a.meshes.n_meshes && gv >= a.meshes.m[mi + 1].vertex_offset) mi++;
    const MeshK& mesh = a.meshes.m[mi];
    const int v = gv - mesh.vertex_offset;
    const float* M = a.link_xf + (size_t(b) * a.meshes.n_meshes + mi) * 48 + 12 * mesh.vertex_link[v];
    const float* p = mesh.vertices + size_t(v) * 3;
    int32_t X, Y;
    project_snap(M, p[0], p[1], p[2], a.cam, X, Y);
    a.snapped[2 * idx] = X;
    a.snapped[2 * idx + 1] = Y;
}

// ---------------------------------------------------------------- workload statistics

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0ull;
}

// Per launch: [0] triangles kept after culling, [1] sum over kept triangles of
// the pixel centres inside their clamped boxes, [2] (triangle, 8x8 block)
// pairs visited, [3] triangles evaluated with 64-bit edge functions.
__global__ __launch_bounds__(256) void stats_kernel(RasterArgs a, unsigned long long* __restrict__ stats) {
    const int b = blockIdx.y;
    __shared__ unsigned long long s_acc[4];
    if (threadIdx.x < 4) s_acc[threadIdx.x] = 0ull;
    __syncthreads();
    unsigned long long kept = 0, pix = 0, pairs = 0, huge = 0;
    for (int mi = 0; mi < a.meshes.n_meshes; mi++) {
        const MeshK& mesh = a.meshes.m[mi];
        const float* M = a.link_xf + (size_t(b) * a.meshes.n_meshes + mi) * 48;
        for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < mesh.n_triangles; t += gridDim.x * blockDim.x) {
            int32_t X[3], Y[3];
            for (int k = 0; k < 3; k++) {
                const int32_t v = mesh.triangles[3 * t + k];
                const float* p = mesh.vertices + size_t(v) * 3;
                project_snap(M + 12 * mesh.vertex_link[v], p[0], p[1], p[2], a.cam, X[k], Y[k]);
            }
            TriRec r;
            if (!setup_triangle(X[0], Y[0], X[1], Y[1], X[2], Y[2], a.cam, r)) continue;
            kept++;
            pairs += uint64_t(r.nbx) * uint64_t(r.nby & 0xffff);
            huge += (r.nby & kHugeBit) ? 1 : 0;
            // exact pixel box from the vertices again
            const int32_t xmin = min(X[0], min(X[1], X[2])), xmax = max(X[0], max(X[1], X[2]));
            const int32_t ymin = min(Y[0], min(Y[1], Y[2])), ymax = max(Y[0], max(Y[1], Y[2]));
            const int32_t px0 = max((xmin - 128 + 255) >> 8, 0), px1 = min((xmax - 128) >> 8, a.cam.width - 1);
            const int32_t py0 = max((ymin - 128 + 255) >> 8, 0), py1 = min((ymax - 128) >> 8, a.cam.height - 1);
            pix += uint64_t(px1 - px0 + 1) * uint64_t(py1 - py0 + 1);
        }
    }
    atomicAdd(&s_acc[0], kept);
    atomicAdd(&s_acc[1], pix);
    atomicAdd(&s_acc[2], pairs);
    atomicAdd(&s_acc[3], huge);
    __syncthreads();
    if (threadIdx.x < 4) atomicAdd(&stats[threadIdx.x], s_acc[threadIdx.x]);
}

// ---------------------------------------------------------------- mask counts

template <bool WITH_TARGET>
__global__ __launch_bounds__(256) void mask_count_kernel(const unsigned long long* __restrict__ masks,
                                                         const unsigned long long* __restrict__ target, CamK cam,
                                                         int32_t* __restrict__ out) {
    __shared__ int32_t s_red[2][4];
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int words = cam.words_x * cam.words_y;
    const unsigned long long* S = masks + size_t(b) * words;
    int32_t cs = 0, ci = 0;
    for (int w = tid; w < words; w += 256) {
        const int wy = w / cam.words_x, wx = w - wy * cam.words_x;
        const unsigned long long v = S[w] & valid_bits(wx, wy, cam);
        cs += __popcll(v);
        if (WITH_TARGET) ci += __popcll(v & target[w]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        cs += __shfl_xor(cs, off);
        ci += __shfl_xor(ci, off);
    }
    if (lane == 0) {
        s_red[0][wave] = cs;
        s_red[1][wave] = ci;
    }
    __syncthreads();
    if (tid == 0) {
        const int32_t ts = s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3];
        const int32_t ti = s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3];
        if (WITH_TARGET) {
            out[2 * b] = ts;
            out[2 * b + 1] = ti;
        } else {
            out[b] = ts;
        }
    }
}

// ---------------------------------------------------------------- host side

size_t mask_lds_bytes(const CamK& cam) { return sizeof(unsigned long long) * size_t(cam.words_x) * cam.words_y; }

constexpr size_t kStaticLds = sizeof(TriRec) * kRasterThreads + sizeof(float) * kMaxArms * 48 + 64;
constexpr size_t kLdsLimit = 160 * 1024;

template <bool FS, bool WM, bool CN>
tk_status launch_raster(const RasterArgs& a, hipStream_t s, const char* what) {
    const size_t lds = mask_lds_bytes(a.cam);
    if (lds + kStaticLds > kLdsLimit)
        return fail(TK_ERR_UNSUPPORTED, "%s: image %dx%d needs %zu bytes of LDS for its mask (limit %zu)", what,
                    a.cam.width, a.cam.height, lds, kLdsLimit - kStaticLds);
    if (a.batch == 0) return TK_OK;
    auto kern = raster_kernel<FS, WM, CN, kRasterThreads>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsLimit - kStaticLds));
    });
    if (attr_err != hipSuccess)
        return fail(TK_ERR_DEVICE, "%s: cannot raise the dynamic LDS limit: %s", what, hipGetErrorString(attr_err));
    hipLaunchKernelGGL(kern, dim3(a.batch), dim3(kRasterThreads), lds, s, a);
    return check_launch(what);
}

tk_status common_raster_checks(int32_t batch, const tk_mesh* meshes, int32_t n_meshes, const tk_camera* cam,
                               RasterArgs* a) {
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    if (tk_status st = validate_camera(cam)) return st;
    if (tk_status st = validate_meshes(meshes, n_meshes, &a->meshes)) return st;
    a->cam = make_cam(*cam);
    a->batch = batch;
    a->link_xf = nullptr;
    a->snapped = nullptr;
    a->masks = nullptr;
    a->target = nullptr;
    a->counts = nullptr;
    return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_raster_silhouette(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                               const tk_camera* cam, uint64_t* d_masks, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &a)) return st;
    TK_REQUIRE(batch == 0 || (d_link_xf && d_masks), "link_xf / masks is NULL");
    a.link_xf = d_link_xf;
    a.masks = reinterpret_cast<unsigned long long*>(d_masks);
    return launch_raster<false, true, false>(a, reinterpret_cast<hipStream_t>(s), "tk_raster_silhouette");
}

tk_status tk_raster_from_snapped(const int32_t* d_snapped, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                                 const tk_camera* cam, uint64_t* d_masks, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &a)) return st;
    TK_REQUIRE(batch == 0 || (d_snapped && d_masks), "snapped / masks is NULL");
    a.snapped = d_snapped;
    a.masks = reinterpret_cast<unsigned long long*>(d_masks);
    return launch_raster<true, true, false>(a, reinterpret_cast<hipStream_t>(s), "tk_raster_from_snapped");
}

tk_status tk_eval_fused(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                        const tk_camera* cam, const uint64_t* d_target, int32_t* d_counts, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &a)) return st;
    TK_REQUIRE(batch == 0 || (d_link_xf && d_target && d_counts), "link_xf / target / counts is NULL");
    a.link_xf = d_link_xf;
    a.target = reinterpret_cast<const unsigned long long*>(d_target);
    a.counts = d_counts;
    return launch_raster<false, false, true>(a, reinterpret_cast<hipStream_t>(s), "tk_eval_fused");
}

tk_status tk_snap_vertices(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                           const tk_camera* cam, int32_t* d_snapped, tk_stream s) {
    clear_error();
    RasterArgs r;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &r)) return st;
    TK_REQUIRE(batch == 0 || (d_link_xf && d_snapped), "link_xf / snapped is NULL");
    if (batch == 0) return TK_OK;
    SnapArgs a{r.meshes, r.cam, d_link_xf, d_snapped, batch};
    const int64_t total = int64_t(batch) * r.meshes.total_vertices;
    const int threads = 256;
    hipLaunchKernelGGL(snap_kernel, dim3(unsigned((total + threads - 1) / threads)), dim3(threads), 0,
                       reinterpret_cast<hipStream_t>(s), a);
    return check_launch("tk_snap_vertices");
}

tk_status tk_mask_loss(const uint64_t* d_masks, int32_t batch, const uint64_t* d_target, const tk_camera* cam,
                       int32_t* d_counts, tk_stream s) {
    clear_error();
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    if (tk_status st = validate_camera(cam)) return st;
    TK_REQUIRE(batch == 0 || (d_masks && d_target && d_counts), "masks / target / counts is NULL");
    if (batch == 0) return TK_OK;
    hipLaunchKernelGGL(mask_count_kernel<true>, dim3(batch), dim3(256), 0, reinterpret_cast<hipStream_t>(s),
                       reinterpret_cast<const unsigned long long*>(d_masks),
                       reinterpret_cast<const unsigned long long*>(d_target), make_cam(*cam), d_counts);
    return check_launch("tk_mask_loss");
}

tk_status tk_mask_popcount(const uint64_t* d_masks, int32_t batch, const tk_camera* cam, int32_t* d_count,
                           tk_stream s) {
    clear_error();
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    if (tk_status st = validate_camera(cam)) return st;
    TK_REQUIRE(batch == 0 || (d_masks && d_count), "masks / count is NULL");
    if (batch == 0) return TK_OK;
    hipLaunchKernelGGL(mask_count_kernel<false>, dim3(batch), dim3(256), 0, reinterpret_cast<hipStream_t>(s),
                       reinterpret_cast<const unsigned long long*>(d_masks), nullptr, make_cam(*cam), d_count);
    return check_launch("tk_mask_popcount");
}

tk_status tk_raster_stats(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                          const tk_camera* cam, uint64_t* d_stats, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &a)) return st;
    TK_REQUIRE(d_stats != nullptr, "stats is NULL");
    TK_REQUIRE(batch == 0 || d_link_xf, "link_xf is NULL");
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s),
                       reinterpret_cast<unsigned long long*>(d_stats), 4);
    if (tk_status st = check_launch("tk_raster_stats")) return st;
    if (batch == 0) return TK_OK;
    a.link_xf = d_link_xf;
    hipLaunchKernelGGL(stats_kernel, dim3(16, batch), dim3(256), 0, reinterpret_cast<hipStream_t>(s), a,
                       reinterpret_cast<unsigned long long*>(d_stats));
    return check_launch("tk_raster_stats");
}

}  // extern "C"
