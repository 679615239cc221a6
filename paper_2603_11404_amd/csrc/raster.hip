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

// 64-byte record of one kept triangle.  The first 48 bytes are all the per-lane
// task path reads.
struct TriRec {
    int32_t e0lo[3];       // low words of the edge functions at the centre of pixel (px0, py0), bias included
    int32_t dx[3], dy[3];  // edge vectors in Q8 units (edge e runs from vertex e to vertex e+1)
    int32_t box_x;         // px0 | px1 << 16  (clamped pixel box)
    int32_t box_y;         // py0 | py1 << 16
    int32_t flags;         // bit 0: 64-bit edge functions; bit 1: near (lane tasks)
    int32_t e0hi[3];       // high words of the edge functions
    int32_t pad;
};
static_assert(sizeof(TriRec) == 64, "record size");

constexpr int32_t kWide = 1;            // flags bit: 64-bit edge functions
constexpr int32_t kNear = 2;            // flags bit: every vertex within 32 px of the box origin (lane tasks)

__device__ __forceinline__ int64_t rec_e0(const TriRec& r, int e) {
    return int64_t((uint64_t(uint32_t(r.e0hi[e])) << 32) | uint64_t(uint32_t(r.e0lo[e])));
}

// Builds the record of one triangle from its snapped vertices; false if culled
// (a vertex before the near plane, zero area, or no pixel centre on screen).
__device__ __forceinline__ bool setup_triangle(int32_t x0, int32_t y0, int32_t x1, int32_t y1, int32_t x2,
                                               int32_t y2, const CamK& cam, TriRec& r) {
    if (x0 == INT32_MIN || x1 == INT32_MIN || x2 == INT32_MIN) return false;
    const int32_t xmin = min(x0, min(x1, x2)), xmax = max(x0, max(x1, x2));
    const int32_t ymin = min(y0, min(y1, y2)), ymax = max(y0, max(y1, y2));
    // pixel centres 256 p + 128 inside [min, max], clamped to the image
    const int32_t px0 = max((xmin - 128 + 255) >> 8, 0), px1 = min((xmax - 128) >> 8, cam.width - 1);
    const int32_t py0 = max((ymin - 128 + 255) >> 8, 0), py1 = min((ymax - 128) >> 8, cam.height - 1);
    if (px0 > px1 || py0 > py1) return false;
    r.box_x = px0 | (px1 << 16);
    r.box_y = py0 | (py1 << 16);
    // vertices relative to the box origin (Q8); near: all within 32 pixels of it
    const int32_t ox = px0 << 8, oy = py0 << 8;
    const bool near = (xmax - ox < (1 << 13)) & (xmin - ox >= -(1 << 13)) & (ymax - oy < (1 << 13)) &
                      (ymin - oy >= -(1 << 13));
    bool wide = false;
    if (near) {
        // differences < 2^14, so all products fit the 24-bit multiplier and every
        // edge function over the box (and 7 pixels beyond it) stays below 2^30 --
        // exact in 32 bits; the high words are never read for near triangles
        int32_t rx[3] = {x0 - ox, x1 - ox, x2 - ox}, ry[3] = {y0 - oy, y1 - oy, y2 - oy};
        const int32_t area2 = __mul24(x1 - x0, y2 - y0) - __mul24(y1 - y0, x2 - x0);
        if (area2 == 0) return false;
        if (area2 < 0) {
            int32_t t = rx[1]; rx[1] = rx[2]; rx[2] = t;
            t = ry[1]; ry[1] = ry[2]; ry[2] = t;
        }
        for (int e = 0; e < 3; e++) {
            const int n = e == 2 ? 0 : e + 1;
            const int32_t dx = rx[n] - rx[e], dy = ry[n] - ry[e];
            const bool top_left = (dy < 0) || (dy == 0 && dx > 0);
            r.e0lo[e] = __mul24(dx, 128 - ry[e]) + __mul24(dy, rx[e] - 128) - (top_left ? 0 : 1);
            r.e0hi[e] = 0;
            r.dx[e] = dx;
            r.dy[e] = dy;
        }
    } else {
        const int32_t w = px1 - px0, h = py1 - py0;
        int32_t vx[3] = {x0, x1, x2}, vy[3] = {y0, y1, y2};
        const int64_t area2 = int64_t(x1 - x0) * int64_t(y2 - y0) - int64_t(y1 - y0) * int64_t(x2 - x0);
        if (area2 == 0) return false;
        if (area2 < 0) {
            vx[1] = x2; vx[2] = x1;
            vy[1] = y2; vy[2] = y1;
        }
        const int64_t cx = int64_t(ox) + 128, cy = int64_t(oy) + 128;
        for (int e = 0; e < 3; e++) {
            const int n = e == 2 ? 0 : e + 1;
            const int32_t dx = vx[n] - vx[e], dy = vy[n] - vy[e];
            const bool top_left = (dy < 0) || (dy == 0 && dx > 0);
            const int64_t E = int64_t(dx) * (cy - vy[e]) - int64_t(dy) * (cx - vx[e]) + (top_left ? 0 : -1);
            r.e0lo[e] = int32_t(uint32_t(uint64_t(E)));
            r.e0hi[e] = int32_t(uint32_t(uint64_t(E) >> 32));
            r.dx[e] = dx;
            r.dy[e] = dy;
            // largest |E| over the pixel centres within 7 pixels of the box
            const int64_t a = int64_t(256) * (dy < 0 ? -int64_t(dy) : int64_t(dy));
            const int64_t b = int64_t(256) * (dx < 0 ? -int64_t(dx) : int64_t(dx));
            const int64_t bound = (E < 0 ? -E : E) + a * (w + 7) + b * (h + 7);
            wide |= bound >= (int64_t(1) << 31);
        }
    }
    r.flags = (wide ? kWide : 0) | (near ? kNear : 0);
    r.pad = 0;
    return true;
}

// ---------------------------------------------------------------- per-wave LDS staging (struct of arrays)

// Slot j's record is four 16-byte groups q0[j]..q3[j]: lanes reading different
// slots read consecutive 16-byte chunks (no bank conflicts), lanes reading one
// slot get a broadcast.
struct WaveStage {
    int4 q0[kWave];   // e0lo[0..2], box_x
    int4 q1[kWave];   // dx[0..2],   box_y
    int4 q2[kWave];   // dy[0..2],   flags
    int4 q3[kWave];   // e0hi[0..2], inclusive prefixes of the lane-task counts (wide | narrow << 16)
    int4 qi[kWave];   // vertex indices of each lane's triangle two chunks ahead
};

__device__ __forceinline__ void stage_put(WaveStage& st, int j, const TriRec& r) {
    st.q0[j] = make_int4(r.e0lo[0], r.e0lo[1], r.e0lo[2], r.box_x);
    st.q1[j] = make_int4(r.dx[0], r.dx[1], r.dx[2], r.box_y);
    st.q2[j] = make_int4(r.dy[0], r.dy[1], r.dy[2], r.flags);
}

__device__ __forceinline__ TriRec stage_get(const WaveStage& st, int j) {
    TriRec r;
    const int4 a = st.q0[j], b = st.q1[j], c = st.q2[j], d = st.q3[j];
    r.e0lo[0] = a.x; r.e0lo[1] = a.y; r.e0lo[2] = a.z; r.box_x = a.w;
    r.dx[0] = b.x; r.dx[1] = b.y; r.dx[2] = b.z; r.box_y = b.w;
    r.dy[0] = c.x; r.dy[1] = c.y; r.dy[2] = c.z; r.flags = c.w;
    r.e0hi[0] = d.x; r.e0hi[1] = d.y; r.e0hi[2] = d.z;
    r.pad = 0;
    return r;
}

// Lane tasks of a near triangle: 8-column windows starting at the box's left
// column, times the 4-row bands (aligned to the mask words) the box touches.
__device__ __forceinline__ int task_windows(int box_x) { return ((box_x >> 16) - (box_x & 0xffff)) / 8 + 1; }
__device__ __forceinline__ int task_bands(int box_y) { return ((box_y >> 16) >> 2) - ((box_y & 0xffff) >> 2) + 1; }

// Narrow near triangles (box at most 2 columns wide, most of a fine mesh's
// slivers) get their own tasks: the 2 box columns times one mask-word row of
// 8 pixel rows.
__device__ __forceinline__ bool is_narrow(int box_x) { return (box_x >> 16) - (box_x & 0xffff) <= 1; }
__device__ __forceinline__ int narrow_tasks(int box_y) { return ((box_y >> 16) >> 3) - ((box_y & 0xffff) >> 3) + 1; }

// Bit r of an 8-bit column mask to bit 8r of a mask word (rows of one column):
// each nibble times 2^0 + 2^7 + 2^14 + 2^21 places its bit i at 8i with no
// two partial products on the same bit, so no carries.
__device__ __forceinline__ unsigned long long spread_column(uint32_t m) {
    const uint32_t lo = ((m & 15u) * 0x204081u) & 0x01010101u;
    const uint32_t hi = (((m >> 4) & 15u) * 0x204081u) & 0x01010101u;
    return (unsigned long long)lo | ((unsigned long long)hi << 32);
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4 and 8
// within each row of 16 lanes, then each row adds the last lane of the rows
// before it (row broadcasts of lanes 15 and 31).  Lanes whose source lies
// outside the row, or whose row is masked off, add 0.
__device__ __forceinline__ int wave_inclusive_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return x;
}

// ---------------------------------------------------------------- coverage of one lane task

// One lane rasterises the part of a near triangle's box inside one window of
// 8 columns x one 4-row band, with incremental 32-bit edge functions, fully
// unrolled: each row tests 8 pixel centres right to left and collects the
// outside flags with v_alignbit.  The 4 row bytes are then split between the
// (at most two) mask words the window straddles and ORed into LDS.
__device__ __forceinline__ void cover_window(const WaveStage& st, int j, int k, unsigned long long* __restrict__ s_mask,
                                             int words_x) {
    const int4 q0 = st.q0[j], q1 = st.q1[j], q2 = st.q2[j];
    const int px0 = q0.w & 0xffff, px1 = q0.w >> 16;
    const int py0 = q1.w & 0xffff, py1 = q1.w >> 16;
    const int nwin = (px1 - px0) / 8 + 1;
    // k = band * nwin + win  (small integers: the float quotient is exact after flooring)
    const int band_i = int(floorf((float(k) + 0.5f) * __builtin_amdgcn_rcpf(float(nwin))));
    const int win = k - band_i * nwin;
    const int band = (py0 >> 2) + band_i;
    const int xa = px0 + 8 * win, xe = min(xa + 7, px1);
    const int ya = max(py0, 4 * band), yb = min(py1, 4 * band + 3);
    const int32_t e0[3] = {q0.x, q0.y, q0.z}, dxs[3] = {q1.x, q1.y, q1.z}, dys[3] = {q2.x, q2.y, q2.z};
    uint32_t A[3], E[3], B[3];
    for (int e = 0; e < 3; e++) {
        const int32_t dx = dxs[e], dy = dys[e];
        A[e] = 0u - (uint32_t(dy) << 8);
        B[e] = uint32_t(dx) << 8;
        E[e] = uint32_t(e0[e] + __mul24(-(dy << 8), xe - px0) + __mul24(dx << 8, ya - py0));
    }
    const int align = 7 - (xe - xa);
    uint32_t rows = 0u;
#pragma unroll
    for (int row = 0; row < 4; row++) {
        uint32_t t0 = E[0], t1 = E[1], t2 = E[2], neg = 0u;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            neg = __builtin_amdgcn_alignbit(neg, t0 | t1 | t2, 31);
            t0 -= A[0];
            t1 -= A[1];
            t2 -= A[2];
        }
        // bit i of neg is pixel xe - 7 + i; after the shift bit c is column xa + c
        const uint32_t cov = (~neg & 0xFFu) >> align;
        if (ya + row <= yb) rows |= cov << (8 * ((ya + row) & 3));
        E[0] += B[0];
        E[1] += B[1];
        E[2] += B[2];
    }
    if (!rows) return;
    const int wx = xa >> 3, sh = xa & 7, wy = band >> 1, half = 32 * (band & 1);
    const uint32_t lo = (rows << sh) & (0x01010101u * ((0xFFu << sh) & 0xFFu));
    const uint32_t hi = (rows >> (8 - sh)) & (0x01010101u * (0xFFu >> (8 - sh)));
    if (lo) atomicOr(&s_mask[wy * words_x + wx], (unsigned long long)lo << half);
    if (hi) atomicOr(&s_mask[wy * words_x + wx + 1], (unsigned long long)hi << half);
}

// One lane rasterises task k of a narrow near triangle: columns px0 and
// px0 + 1 (the second only if inside the box) over mask-word row
// (py0 >> 3) + k, with incremental 32-bit edge functions (all 8 rows lie
// within 7 pixels of the box, where near triangles' edge functions are exact
// in 32 bits).  Each column's 8 rows are collected with v_alignbit, clipped to
// the box rows, spread to the word's bit layout and ORed into LDS (one word,
// or two when px0 is the last column of a word).
__device__ __forceinline__ void cover_narrow(const WaveStage& st, int j, int k, unsigned long long* __restrict__ s_mask,
                                             int words_x) {
    const int4 q0 = st.q0[j], q1 = st.q1[j], q2 = st.q2[j];
    const int px0 = q0.w & 0xffff, px1 = q0.w >> 16;
    const int py0 = q1.w & 0xffff, py1 = q1.w >> 16;
    const int wy = (py0 >> 3) + k;
    const int32_t e0[3] = {q0.x, q0.y, q0.z}, dxs[3] = {q1.x, q1.y, q1.z}, dys[3] = {q2.x, q2.y, q2.z};
    uint32_t A[3], B[3], E[3];
    for (int e = 0; e < 3; e++) {
        A[e] = 0u - (uint32_t(dys[e]) << 8);          // one column to the right
        B[e] = uint32_t(dxs[e]) << 8;                 // one row down
        E[e] = uint32_t(e0[e] + __mul24(dxs[e] << 8, 8 * wy + 7 - py0));   // bottom row of the word
    }
    // alignbit shifts the flags left and brings the new sign bit in at bit 0:
    // walking the rows bottom-up leaves row 8 wy + r at bit r
    uint32_t neg0 = 0u, neg1 = 0u;
#pragma unroll
    for (int row = 7; row >= 0; row--) {
        neg0 = __builtin_amdgcn_alignbit(neg0, E[0] | E[1] | E[2], 31);
        neg1 = __builtin_amdgcn_alignbit(neg1, (E[0] + A[0]) | (E[1] + A[1]) | (E[2] + A[2]), 31);
        E[0] -= B[0];
        E[1] -= B[1];
        E[2] -= B[2];
    }
    const int lo = max(py0 - 8 * wy, 0), hi = min(py1 - 8 * wy, 7);
    const uint32_t rowmask = (0xFFu << lo) & (0xFFu >> (7 - hi));
    const uint32_t m0 = ~neg0 & rowmask;
    const uint32_t m1 = px1 > px0 ? ~neg1 & rowmask : 0u;
    const int wx = px0 >> 3, sh = px0 & 7;
    unsigned long long w0 = spread_column(m0) << sh;
    if (sh < 7) w0 |= spread_column(m1) << (sh + 1);
    if (w0) atomicOr(&s_mask[wy * words_x + wx], w0);
    if (sh == 7 && m1) atomicOr(&s_mask[wy * words_x + wx + 1], spread_column(m1));
}

// ---------------------------------------------------------------- cooperative coverage of a big triangle

// The whole wave walks the 8x8 blocks of one triangle's box: lane = pixel,
// three edge functions per lane, the 64-lane ballot is the block's word.
__device__ __forceinline__ void cover_big(const WaveStage& st, int j, int lx, int ly, int lane,
                                          unsigned long long* __restrict__ s_mask, int words_x) {
    const TriRec r = stage_get(st, j);
    const int box_x = __builtin_amdgcn_readfirstlane(r.box_x);
    const int box_y = __builtin_amdgcn_readfirstlane(r.box_y);
    const int flags = __builtin_amdgcn_readfirstlane(r.flags);
    const int px0 = box_x & 0xffff, px1 = box_x >> 16, py0 = box_y & 0xffff, py1 = box_y >> 16;
    const int bx0 = px0 >> 3, by0 = py0 >> 3;
    const int nbx = (px1 >> 3) - bx0 + 1, nby = (py1 >> 3) - by0 + 1;
    const int ox = 8 * bx0 + lx - px0, oy = 8 * by0 + ly - py0;   // lane pixel offset from the box origin
    if (!(flags & kWide)) {
        // 32-bit modular evaluation, exact since every |E| over the blocks is < 2^31
        uint32_t L[3], SX[3], SY[3];
        for (int e = 0; e < 3; e++) {
            const uint32_t A = 0u - (uint32_t(r.dy[e]) << 8);
            const uint32_t B = uint32_t(r.dx[e]) << 8;
            L[e] = uint32_t(r.e0lo[e]) + A * uint32_t(ox) + B * uint32_t(oy);
            SX[e] = A * 8u;
            SY[e] = B * 8u;
        }
        for (int by = 0; by < nby; by++) {
            uint32_t E0 = L[0], E1 = L[1], E2 = L[2];
            for (int bx = 0; bx < nbx; bx++) {
                const unsigned long long m = __ballot(int32_t(E0 | E1 | E2) >= 0);
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
        int64_t e0[3];
        for (int e = 0; e < 3; e++) e0[e] = rec_e0(r, e);
        for (int by = 0; by < nby; by++) {
            for (int bx = 0; bx < nbx; bx++) {
                const int64_t px = 8 * bx + ox, py = 8 * by + oy;
                bool in = true;
                for (int e = 0; e < 3; e++) {
                    const int64_t E = e0[e] - int64_t(256) * r.dy[e] * px + int64_t(256) * r.dx[e] * py;
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
    int32_t pretransform;        // snapped points to a workspace the kernel fills first
};

template <bool FROM_SNAPPED, bool WRITE_MASK, bool COUNTS, int NT>
__global__ __launch_bounds__(NT) void raster_kernel(RasterArgs a) {
    constexpr int NW = NT / kWave;
    extern __shared__ unsigned long long s_mask[];
    __shared__ WaveStage s_stage[NW];
    __shared__ float s_M[kMaxArms * 48];
    __shared__ int32_t s_red[2][NW];

    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int lx = lane & 7, ly = lane >> 3;
    const CamK& cam = a.cam;
    const int words = cam.words_x * cam.words_y;
    WaveStage& st = s_stage[wave];

    for (int w = tid; w < words; w += NT) s_mask[w] = 0ull;
    if (!FROM_SNAPPED || a.pretransform)
        for (int i = tid; i < a.meshes.n_meshes * 48; i += NT)
            s_M[i] = a.link_xf[size_t(b) * a.meshes.n_meshes * 48 + i];
    __syncthreads();
    if (FROM_SNAPPED && a.pretransform) {
        // transform, project and snap every vertex of this candidate once into the workspace
        int2* out = reinterpret_cast<int2*>(const_cast<int32_t*>(a.snapped)) + size_t(b) * a.meshes.total_vertices;
        for (int mi = 0; mi < a.meshes.n_meshes; mi++) {
            const MeshK& mesh = a.meshes.m[mi];
            for (int v = tid; v < mesh.n_vertices; v += NT) {
                const float* p = mesh.vertices + size_t(v) * 3;
                int32_t X, Y;
                project_snap(s_M + mi * 48 + 12 * mesh.vertex_link[v], p[0], p[1], p[2], cam, X, Y);
                out[mesh.vertex_offset + v] = make_int2(X, Y);
            }
        }
        __syncthreads();
    }

    for (int mi = 0; mi < a.meshes.n_meshes; mi++) {
        const MeshK& mesh = a.meshes.m[mi];
        const float* M = s_M + mi * 48;
        const int T = mesh.n_triangles;
        const int2* snap = reinterpret_cast<const int2*>(a.snapped) +
                           (size_t(b) * a.meshes.total_vertices + mesh.vertex_offset);
        // Software pipeline over the wave's chunks of 64 triangles: while chunk c
        // is processed, the snapped vertices of chunk c + 1 and the indices of
        // chunk c + 2 are in flight (the vertex gathers are the long-latency
        // loads).  Without snapped input, indices run one chunk ahead.
        // The indices loaded for chunk c + 2 are parked in the wave's LDS stage
        // at the end of the iteration: kept in registers across the loop they
        // would be moved right after their load, and that move would wait for
        // the vertex gathers issued just before.
        const int3* tri3 = reinterpret_cast<const int3*>(mesh.triangles);
        int t = wave * kWave + lane;
        int32_t idx[3] = {0, 0, 0};
        int2 pv[3] = {make_int2(INT32_MIN, 0), make_int2(INT32_MIN, 0), make_int2(INT32_MIN, 0)};
        if (FROM_SNAPPED) {
            if (t < T) {
                const int3 i0 = tri3[t];
                pv[0] = snap[i0.x];
                pv[1] = snap[i0.y];
                pv[2] = snap[i0.z];
            }
            if (t + NT < T) {
                const int3 i1 = tri3[t + NT];
                st.qi[lane] = make_int4(i1.x, i1.y, i1.z, 0);
            }
        } else if (t < T) {
            for (int k = 0; k < 3; k++) idx[k] = mesh.triangles[3 * t + k];
        }
        for (int base = wave * kWave; base < T; base += NT) {
            t = base + lane;
            const bool live = t < T;
            int32_t X[3] = {INT32_MIN, INT32_MIN, INT32_MIN}, Y[3] = {0, 0, 0};
            float vx[3], vy[3], vz[3];
            int link[3];
            int3 ahead;
            if (FROM_SNAPPED) {
                if (live)
                    for (int k = 0; k < 3; k++) {
                        X[k] = pv[k].x;
                        Y[k] = pv[k].y;
                    }
                if (t + NT < T) {
                    const int4 q = st.qi[lane];
                    pv[0] = snap[q.x];
                    pv[1] = snap[q.y];
                    pv[2] = snap[q.z];
                }
                ahead = tri3[min(t + 2 * NT, T - 1)];   // unconditional: no initialised registers to guard
            } else {
                if (live)
                    for (int k = 0; k < 3; k++) {
                        const float* v = mesh.vertices + size_t(idx[k]) * 3;
                        vx[k] = v[0];
                        vy[k] = v[1];
                        vz[k] = v[2];
                        link[k] = mesh.vertex_link[idx[k]];
                    }
                // prefetch the next chunk's indices while this chunk is processed
                const int tn = t + NT;
                if (tn < T)
                    for (int k = 0; k < 3; k++) idx[k] = mesh.triangles[3 * tn + k];
            }
            if (!FROM_SNAPPED && live)
                for (int k = 0; k < 3; k++) project_snap(M + 12 * link[k], vx[k], vy[k], vz[k], cam, X[k], Y[k]);
            TriRec rec;
            const bool valid = live && setup_triangle(X[0], Y[0], X[1], Y[1], X[2], Y[2], cam, rec);
            const bool near = valid && (rec.flags & kNear);
            const bool narrow = near && is_narrow(rec.box_x);
            if (valid) stage_put(st, lane, rec);
            // lane tasks of near triangles: 8-column windows x 4-row bands (at
            // most 5 x 9 each) for wide boxes, word rows (at most 6) for narrow
            // ones; inclusive prefixes over the wave from one ballot per bit
            const int cnt = near && !narrow ? task_windows(rec.box_x) * task_bands(rec.box_y) : 0;
            const int cnt_n = narrow ? narrow_tasks(rec.box_y) : 0;
            // both counts in one scan: wide in the low, narrow in the high 16 bits
            // (totals stay below 64 x 45)
            const int incl_both = wave_inclusive_sum(cnt | (cnt_n << 16));
            const int total_both = __builtin_amdgcn_readlane(incl_both, kWave - 1);
            const int total = total_both & 0xffff, total_n = total_both >> 16;
            st.q3[lane] = make_int4(rec.e0hi[0], rec.e0hi[1], rec.e0hi[2], incl_both);
            const unsigned long long big = __ballot(valid && !near);
            // staged fields written by other lanes must be visible before they are read
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

            for (int base = 0; base < total_n; base += kWave) {
                const int q = base + lane;
                if (q < total_n) {
                    int j = 0;
#pragma unroll
                    for (int step = kWave / 2; step > 0; step >>= 1)
                        if ((st.q3[j + step - 1].w >> 16) <= q) j += step;
                    const int k = q - ((st.q3[j].w >> 16) - narrow_tasks(st.q1[j].w));
                    cover_narrow(st, j, k, s_mask, cam.words_x);
                }
            }
            for (int base = 0; base < total; base += kWave) {
                const int q = base + lane;
                if (q < total) {
                    // slot j: first lane whose inclusive prefix exceeds q
                    int j = 0;
#pragma unroll
                    for (int step = kWave / 2; step > 0; step >>= 1)
                        if ((st.q3[j + step - 1].w & 0xffff) <= q) j += step;
                    const int k = q - ((st.q3[j].w & 0xffff) - task_windows(st.q0[j].w) * task_bands(st.q1[j].w));
                    cover_window(st, j, k, s_mask, cam.words_x);
                }
            }
            unsigned long long todo = big;
            while (todo) {
                const int j = __builtin_ctzll(todo);
                todo &= todo - 1;
                cover_big(st, j, lx, ly, lane, s_mask, cam.words_x);
            }
            if (FROM_SNAPPED && t + 2 * NT < T) st.qi[lane] = make_int4(ahead.x, ahead.y, ahead.z, 0);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
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
            {
                const int bx0 = (r.box_x & 0xffff) >> 3, bx1 = (r.box_x >> 16) >> 3;
                const int by0 = (r.box_y & 0xffff) >> 3, by1 = (r.box_y >> 16) >> 3;
                pairs += uint64_t(bx1 - bx0 + 1) * uint64_t(by1 - by0 + 1);
            }
            huge += (r.flags & kWide) ? 1 : 0;
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

constexpr size_t kLdsLimit = 160 * 1024;

template <int NT>
constexpr size_t static_lds() {
    return sizeof(WaveStage) * (NT / kWave) + sizeof(float) * kMaxArms * 48 + sizeof(int32_t) * 2 * (NT / kWave);
}

template <bool FS, bool WM, bool CN, int NT>
tk_status launch_raster_nt(const RasterArgs& a, size_t lds, hipStream_t s, const char* what) {
    auto kern = raster_kernel<FS, WM, CN, NT>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kLdsLimit - static_lds<NT>()));
    });
    if (attr_err != hipSuccess)
        return fail(TK_ERR_DEVICE, "%s: cannot raise the dynamic LDS limit: %s", what, hipGetErrorString(attr_err));
    hipLaunchKernelGGL(kern, dim3(a.batch), dim3(NT), lds, s, a);
    return check_launch(what);
}

// One workgroup per candidate; the widest block (16, 8 or 4 waves) whose
// staging fits in LDS next to the image mask.
template <bool FS, bool WM, bool CN>
tk_status launch_raster(const RasterArgs& a, hipStream_t s, const char* what) {
    const size_t lds = mask_lds_bytes(a.cam);
    if (lds + static_lds<256>() > kLdsLimit)
        return fail(TK_ERR_UNSUPPORTED, "%s: image %dx%d needs %zu bytes of LDS for its mask (limit %zu)", what,
                    a.cam.width, a.cam.height, lds, kLdsLimit - static_lds<256>());
    if (a.batch == 0) return TK_OK;
    if (lds + static_lds<1024>() <= kLdsLimit) return launch_raster_nt<FS, WM, CN, 1024>(a, lds, s, what);
    if (lds + static_lds<512>() <= kLdsLimit) return launch_raster_nt<FS, WM, CN, 512>(a, lds, s, what);
    return launch_raster_nt<FS, WM, CN, 256>(a, lds, s, what);
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
    a->pretransform = 0;
    return TK_OK;
}

// With a workspace of batch * sum(V) * 8 bytes the kernel snaps every vertex
// once into it and rasterises from there; without one each triangle
// transforms its own three vertices.
tk_status attach_workspace(RasterArgs* a, void* d_ws, size_t ws_bytes, const char* what) {
    if (d_ws == nullptr) return TK_OK;
    const size_t need = size_t(a->batch) * size_t(a->meshes.total_vertices) * 2 * sizeof(int32_t);
    if (ws_bytes < need)
        return fail(TK_ERR_WORKSPACE_TOO_SMALL, "%s: workspace of %zu bytes, %zu needed", what, ws_bytes, need);
    TK_REQUIRE((reinterpret_cast<uintptr_t>(d_ws) & 7) == 0, "%s: workspace must be 8-byte aligned", what);
    a->snapped = static_cast<const int32_t*>(d_ws);
    a->pretransform = 1;
    return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

size_t tk_raster_workspace_bytes(int32_t batch, const tk_mesh* meshes, int32_t n_meshes) {
    if (batch < 0 || meshes == nullptr || n_meshes < 1 || n_meshes > kMaxArms) return 0;
    size_t v = 0;
    for (int i = 0; i < n_meshes; i++) v += size_t(meshes[i].n_vertices > 0 ? meshes[i].n_vertices : 0);
    return size_t(batch) * v * 2 * sizeof(int32_t);
}

tk_status tk_raster_silhouette(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                               const tk_camera* cam, uint64_t* d_masks, void* d_ws, size_t ws_bytes, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &a)) return st;
    TK_REQUIRE(batch == 0 || (d_link_xf && d_masks), "link_xf / masks is NULL");
    a.link_xf = d_link_xf;
    a.masks = reinterpret_cast<unsigned long long*>(d_masks);
    if (tk_status st = attach_workspace(&a, d_ws, ws_bytes, "tk_raster_silhouette")) return st;
    if (a.pretransform)
        return launch_raster<true, true, false>(a, reinterpret_cast<hipStream_t>(s), "tk_raster_silhouette");
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
                        const tk_camera* cam, const uint64_t* d_target, int32_t* d_counts, void* d_ws,
                        size_t ws_bytes, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = common_raster_checks(batch, meshes, n_meshes, cam, &a)) return st;
    TK_REQUIRE(batch == 0 || (d_link_xf && d_target && d_counts), "link_xf / target / counts is NULL");
    a.link_xf = d_link_xf;
    a.target = reinterpret_cast<const unsigned long long*>(d_target);
    a.counts = d_counts;
    if (tk_status st = attach_workspace(&a, d_ws, ws_bytes, "tk_eval_fused")) return st;
    if (a.pretransform) return launch_raster<true, false, true>(a, reinterpret_cast<hipStream_t>(s), "tk_eval_fused");
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
