// Binary silhouette rasterisation and mask counts on gfx950 (wave64).
//
// Renderer S = R(K(Pi(T_r^c T_m^r(q) v_m))) of paper Sec. III-A.2 with
// S in {0,1}^{H x W}; counts |S| and |S and M_ref| feed the render loss
// (Eq. render_loss) and the mask error 1 - IoU (Sec. IV).
//
// Design (one workgroup per candidate, its whole image mask in LDS as 8x8-pixel
// u64 words):
//   0. (ask-eval form) wave 0 draws the candidate from the CMA-ES state and
//      evaluates its forward kinematics into LDS; the other waves clear the mask;
//   1. (with a workspace) every vertex of the candidate is transformed (FP32, no
//      contraction), tested against the near plane, projected and snapped to Q8
//      once, into the workspace;
//   2. triangles are numbered in chunks of 64 over all meshes; each wave starts
//      on two chunks and claims later ones from an LDS counter, loading indices
//      and snapped vertices ahead of use.  Each lane sets up one triangle: cull
//      (flagged vertex, zero area, empty box; for a closed mesh whose vertices
//      all passed the near plane, negative area too, since its positively
//      oriented triangles alone cover the same pixel centres), orientation,
//      exact integer edge functions E(p) = dx (p.y - y0) - dy (p.x - x0) at
//      pixel centres with the top-left bias, the pixel box;
//   3. small-box triangles (32-bit arithmetic) become lane tasks in two per-wave
//      LDS ring queues (narrow boxes: 2 columns x 6 rows per task; wide boxes:
//      8 columns x 4 rows), run in rounds of 64 tasks; each task updates its
//      edge functions incrementally and ORs its covered pixels into at most
//      2 x 2 mask words; triangles needing 64-bit edge functions are covered by
//      the whole wave, 8x8 block by block, each block's word a 64-lane ballot;
//   4. the mask is counted (|S|, |S and M|) against the target with popcounts
//      and/or written out.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "fitness_device.h"
#include "sample_device.h"

namespace tk {
namespace {

constexpr int kWave = 64;

// ---------------------------------------------------------------- vertex transform

// FP32 transform p = M [v; 1], pinhole projection and Q8 snap (round half to
// even).  Returns false when the vertex is culled (Z < z_near or NaN).  Every
// form of the raster path calls this one function, so they snap identically.
// The transform rows are three explicit fused multiply-adds each, and the
// perspective divide is one hardware reciprocal (1 ulp) and two products,
// within 3 ulp of the quotients: all far inside the FP32 bound of the
// transform.
__device__ __forceinline__ bool project_snap(const float* __restrict__ M, float vx, float vy, float vz,
                                             const CamK& cam, int32_t& X, int32_t& Y) {
#pragma clang fp contract(off)
    const float px = fmaf(M[0], vx, fmaf(M[1], vy, fmaf(M[2], vz, M[3])));
    const float py = fmaf(M[4], vx, fmaf(M[5], vy, fmaf(M[6], vz, M[7])));
    const float pz = fmaf(M[8], vx, fmaf(M[9], vy, fmaf(M[10], vz, M[11])));
    const float rz = __builtin_amdgcn_rcpf(pz);
    float u = fmaf(cam.fx, px * rz, cam.cx);
    float v = fmaf(cam.fy, py * rz, cam.cy);
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
constexpr int32_t kNear = 2;            // flags bit: every vertex within 56 px of the box origin (lane tasks)

// Near triangles have every vertex within kNearQ8 (56 pixels in Q8 units) of
// their box origin.  Then every edge vector is below 2 kNearQ8 = 28672 (it
// packs into 16 bits, and 256 times it fits the 24-bit multiplier), and every
// edge function over the box and 7 pixels beyond it -- the pixel centres the
// lane tasks evaluate -- is below 2 x 28672 x (28672 + 7 x 256) < 1.75e9 <
// 2^31 in magnitude: exact in 32-bit modular arithmetic.
constexpr int32_t kNearQ8 = 56 * 256;

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
    // vertices relative to the box origin (Q8); near: all within 56 pixels of it
    const int32_t ox = px0 << 8, oy = py0 << 8;
    const bool near = (xmax - ox < kNearQ8) & (xmin - ox >= -kNearQ8) & (ymax - oy < kNearQ8) &
                      (ymin - oy >= -kNearQ8);
    bool wide = false;
    if (near) {
        // differences < 2 kNearQ8, so all products fit the 24-bit multiplier and
        // every edge function over the box (and 7 pixels beyond it) is exact in
        // 32 bits (see kNearQ8); the high words are never read for near triangles
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

// Orders this wave's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- per-wave task queues in LDS

// A near triangle's record for the lane tasks, 32 bytes: a = the three edge
// functions at the centre of pixel (px0, py0) (bias included) and the packed
// columns of the box; b = the edge vectors as 16-bit pairs (dx low, dy high:
// a near triangle's edges are shorter than 2^14 in Q8 units) and the packed
// rows of the box.
struct NearRec {
    int4 a, b;
};

__device__ __forceinline__ NearRec pack_near(const TriRec& r) {
    NearRec p;
    p.a = make_int4(r.e0lo[0], r.e0lo[1], r.e0lo[2], r.box_x);
    int32_t d[3];
    for (int e = 0; e < 3; e++) d[e] = int32_t((uint32_t(r.dx[e]) & 0xffffu) | (uint32_t(r.dy[e]) << 16));
    p.b = make_int4(d[0], d[1], d[2], r.box_y);
    return p;
}
__device__ __forceinline__ int32_t rec_dx(int32_t v) { return int32_t(int16_t(v & 0xffff)); }
__device__ __forceinline__ int32_t rec_dy(int32_t v) { return v >> 16; }

// Each wave queues the records of its near triangles -- narrow and wide boxes
// separately -- and runs a round of lane tasks only once 64 tasks of a class
// are pending, so rounds run with every lane busy whatever the mix of the
// chunk.  The queues are rings indexed by running slot counts; start[] holds
// each queued triangle's first task number (a running count of the wave's
// tasks of that class).  A ring is drained (its pending tasks, fewer than 64,
// run as a partial round) before new triangles would overflow it; with 128
// narrow slots that never happens (at most 63 pending plus 64 new).
constexpr int kNarrowRing = 128;
constexpr int kWideRing = 64;
struct WaveQueues {
    int4 na[kNarrowRing], nb[kNarrowRing];
    int32_t nstart[kNarrowRing];
    int4 wa[kWideRing], wb[kWideRing];
    int32_t wstart[kWideRing];
    int32_t mark[64];      // per round: where each queued triangle's tasks start
};

// Bytes of one wave's queues with a narrow ring of nr slots (the layout of
// WaveQueues with kNarrowRing = nr).
__host__ __device__ constexpr int queue_bytes(int nr) { return nr * 36 + kWideRing * 36 + 64 * 4; }
static_assert(queue_bytes(kNarrowRing) == sizeof(WaveQueues), "queue layout");
static_assert(queue_bytes(64) >= 3328, "the ask prologue borrows wave 0's queues as 3.2 KB of scratch");

// One wave's queues inside a block of LDS laid out as WaveQueues with a
// narrow ring of nmask + 1 slots.
struct QueueView {
    int4 *na, *nb, *wa, *wb;
    int32_t *nstart, *wstart, *mark;
    int nmask;   // narrow ring slots - 1
};

__device__ __forceinline__ QueueView queue_view(char* base, int nr) {
    QueueView q;
    q.na = reinterpret_cast<int4*>(base);
    q.nb = q.na + nr;
    q.nstart = reinterpret_cast<int32_t*>(q.nb + nr);
    q.wa = reinterpret_cast<int4*>(q.nstart + nr);
    q.wb = q.wa + kWideRing;
    q.wstart = reinterpret_cast<int32_t*>(q.wb + kWideRing);
    q.mark = q.wstart + kWideRing;
    q.nmask = nr - 1;
    return q;
}

// Lane tasks of a near triangle: 8-column windows times 4-row bands, both
// starting at the box's top-left pixel.
__device__ __forceinline__ int task_windows(int box_x) { return ((box_x >> 16) - (box_x & 0xffff)) / 8 + 1; }
__device__ __forceinline__ int task_bands(int box_y) { return ((box_y >> 16) - (box_y & 0xffff)) / 4 + 1; }

// Narrow near triangles (box at most 2 columns wide, most of a fine mesh's
// slivers) get their own tasks: the 2 box columns times kNarrowRows pixel rows.
__device__ __forceinline__ bool is_narrow(int box_x) { return (box_x >> 16) - (box_x & 0xffff) <= 1; }
// Rows per narrow task.  Narrow boxes of a fine mesh are mostly 1-6 rows tall
// (about 90% at most 4 on the 640x480 instrument, a longer tail at 960x540):
// 6-row tasks leave fewer idle rows than 8-row ones without the extra tasks
// that 4-row ones need for the taller boxes.
constexpr int kNarrowRows = 6;
__device__ __forceinline__ int narrow_tasks(int box_y) {
    return ((box_y >> 16) - (box_y & 0xffff)) / kNarrowRows + 1;
}

// ORs an 8x8 pixel block, bit 8r + c = pixel (xa + c, ya + r), into the (at
// most 2 x 2) mask words it overlaps.  Only pixels inside the image may be set.
__device__ __forceinline__ void or_block(unsigned long long* __restrict__ s_mask, int words_x, int xa, int ya,
                                         unsigned long long bits) {
    const int wx = xa >> 3, sx = xa & 7, wy = ya >> 3, sy = ya & 7;
    const unsigned long long rows[2] = {bits << (8 * sy), sy ? bits >> (64 - 8 * sy) : 0ull};
    const unsigned long long keep = 0x0101010101010101ull * (0xFFull >> sx);         // columns that stay
    const unsigned long long carry = 0x0101010101010101ull * ((1ull << sx) - 1ull);  // columns that move on
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const unsigned long long w0 = (rows[h] & keep) << sx;
        const unsigned long long w1 = (rows[h] >> (8 - sx)) & carry;
        if (w0) atomicOr(&s_mask[(wy + h) * words_x + wx], w0);
        if (w1) atomicOr(&s_mask[(wy + h) * words_x + wx + 1], w1);
    }
}

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

// Inclusive prefix maximum over the 64 lanes (same pattern; absent sources give -1).
__device__ __forceinline__ int wave_inclusive_max(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));   // row_shr:1
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));   // row_shr:2
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));   // row_shr:4
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));   // row_shr:8
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xa, 0xf, false));   // row_bcast:15 into rows 1, 3
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xc, 0xf, false));   // row_bcast:31 into rows 2, 3
    return x;
}

// ---------------------------------------------------------------- coverage of one lane task

// One lane rasterises the part of a near triangle's box inside one window of
// 8 columns x 4 rows (windows and bands start at the box's top-left pixel),
// with incremental 32-bit edge functions, fully unrolled: each row tests 8
// pixel centres right to left and collects the outside flags with
// v_alignbit.  The row bytes are ORed into the (at most 2 x 2) mask words the
// window overlaps.
__device__ __forceinline__ void cover_window(const int4 q0, const int4 q1, int k, unsigned long long* __restrict__ s_mask,
                                             int words_x) {
    const int px0 = q0.w & 0xffff, px1 = q0.w >> 16;
    const int py0 = q1.w & 0xffff, py1 = q1.w >> 16;
    const int nwin = (px1 - px0) / 8 + 1;
    // k = band * nwin + win  (small integers: the float quotient is exact after flooring)
    const int band_i = int(floorf((float(k) + 0.5f) * __builtin_amdgcn_rcpf(float(nwin))));
    const int win = k - band_i * nwin;
    const int xa = px0 + 8 * win, xe = min(xa + 7, px1);
    const int ya = py0 + 4 * band_i, yb = min(py1, ya + 3);
    const int32_t e0[3] = {q0.x, q0.y, q0.z};
    const int32_t dxs[3] = {rec_dx(q1.x), rec_dx(q1.y), rec_dx(q1.z)}, dys[3] = {rec_dy(q1.x), rec_dy(q1.y), rec_dy(q1.z)};
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
        if (ya + row <= yb) rows |= cov << (8 * row);
        E[0] += B[0];
        E[1] += B[1];
        E[2] += B[2];
    }
    if (rows) or_block(s_mask, words_x, xa, ya, rows);
}

// One lane rasterises task k of a narrow near triangle: columns px0 and
// px0 + 1 (the second only if inside the box) over the kNarrowRows pixel rows
// from py0 + kNarrowRows k, with incremental 32-bit edge functions (all rows
// lie within kNarrowRows - 1 pixels of the box, where near triangles' edge
// functions are exact in 32 bits).  Each column's rows are collected with
// v_alignbit, clipped to the box, spread to the block layout and ORed into
// the mask words.
__device__ __forceinline__ void cover_narrow(const int4 q0, const int4 q1, int k, unsigned long long* __restrict__ s_mask,
                                             int words_x) {
    const int px0 = q0.w & 0xffff, px1 = q0.w >> 16;
    const int py0 = q1.w & 0xffff, py1 = q1.w >> 16;
    const int ya = py0 + kNarrowRows * k;
    const int32_t e0[3] = {q0.x, q0.y, q0.z};
    const int32_t dxs[3] = {rec_dx(q1.x), rec_dx(q1.y), rec_dx(q1.z)}, dys[3] = {rec_dy(q1.x), rec_dy(q1.y), rec_dy(q1.z)};
    uint32_t A[3], B[3], E[3];
    for (int e = 0; e < 3; e++) {
        A[e] = 0u - (uint32_t(dys[e]) << 8);          // one column to the right
        B[e] = uint32_t(dxs[e]) << 8;                 // one row down
        E[e] = uint32_t(e0[e] + __mul24(dxs[e] << 8, kNarrowRows * k + kNarrowRows - 1));   // bottom row of the window
    }
    // alignbit shifts the flags left and brings the new sign bit in at bit 0:
    // walking the rows bottom-up leaves row ya + r at bit r
    uint32_t neg0 = 0u, neg1 = 0u;
#pragma unroll
    for (int row = kNarrowRows - 1; row >= 0; row--) {
        neg0 = __builtin_amdgcn_alignbit(neg0, E[0] | E[1] | E[2], 31);
        neg1 = __builtin_amdgcn_alignbit(neg1, (E[0] + A[0]) | (E[1] + A[1]) | (E[2] + A[2]), 31);
        E[0] -= B[0];
        E[1] -= B[1];
        E[2] -= B[2];
    }
    const uint32_t rowmask = (0xFFu >> (8 - kNarrowRows)) >> (kNarrowRows - 1 - min(py1 - ya, kNarrowRows - 1));
    const uint32_t m0 = ~neg0 & rowmask;
    const uint32_t m1 = px1 > px0 ? ~neg1 & rowmask : 0u;
    const unsigned long long bits = spread_column(m0) | (spread_column(m1) << 1);
    if (bits) or_block(s_mask, words_x, px0, ya, bits);
}

// ---------------------------------------------------------------- cooperative coverage of a big triangle

// The whole wave walks the 8x8 blocks of one triangle's box (record r, the
// same in every lane): lane = pixel, three edge functions per lane, the
// 64-lane ballot is the block's word.
__device__ __forceinline__ void cover_big(const TriRec& r, int lx, int ly, int lane,
                                          unsigned long long* __restrict__ s_mask, int words_x) {
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

// ---------------------------------------------------------------- task rounds

// Runs lane tasks done .. done + count - 1 (count <= 64, task done + i on lane
// i) of a queue whose triangles occupy running slots tail .. head - 1 (the
// triangle at tail holds task done).  Lane l marks, in the wave's mark row,
// the lane where triangle tail + l's tasks begin within the round (tail's own
// at lane 0; first-task numbers increase, so marks never collide); a prefix
// maximum over the lanes then gives each lane the last triangle starting at or
// before its task.  Returns the running slot of the triangle that holds task
// done + 64 (the new tail after a full round).
template <bool NARROW>
__device__ __forceinline__ int run_round(const int4* __restrict__ qa, const int4* __restrict__ qb,
                                         const int32_t* __restrict__ qstart, int32_t* __restrict__ mark, int ring_mask,
                                         int tail, int head, int done, int count, int lane,
                                         unsigned long long* __restrict__ s_mask, int words_x) {
    const int q = done + lane;
    int next = tail;
    mark[lane] = -1;
    wave_sync();
    if (lane < head - tail) {
        const int rel = qstart[(tail + lane) & ring_mask] - done;
        if (rel < kWave) mark[max(rel, 0)] = lane;
    }
    wave_sync();
    const int lo = wave_inclusive_max(mark[lane]);   // slot tail + lo starts at or before task q
    if (lane < count) {
        const int slot = (tail + lo) & ring_mask;
        const int k = q - qstart[slot];
        const int4 a = qa[slot], b = qb[slot];
        int ntask;
        if (NARROW) {
            cover_narrow(a, b, k, s_mask, words_x);
            ntask = narrow_tasks(b.w);
        } else {
            cover_window(a, b, k, s_mask, words_x);
            ntask = task_windows(a.w) * task_bands(b.w);
        }
        next = tail + lo + (k == ntask - 1 ? 1 : 0);
    }
    return __builtin_amdgcn_readlane(next, kWave - 1);
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
    // ask-eval form: each workgroup first draws its CMA-ES candidate and
    // evaluates its forward kinematics (link transforms written to link_xf_out)
    int32_t ask;
    int32_t n, lam;
    void* state;
    FkArgs fk;
    float* X;                    // [batch][n]
    float* link_xf_out;          // [batch][n_meshes][4][12]
    float* kp;                   // nullable [batch][n_meshes][4][2]
};

// Ask-eval prologue, run by wave 0 of workgroup b: candidate b of the current
// generation is drawn exactly as the sample kernel draws it (same generator,
// same factor L and arithmetic), written to X and the state's Z and Y, and
// its forward kinematics (same device function as the FK kernel) goes to the
// LDS transforms s_M and to kp; the lane's coordinates are returned for
// ask_store.  When the state already holds this generation's z (drawn by the
// previous update), they are read instead of drawn.  scratch: >= 3.2 KB of
// LDS.
struct AskOut {
    double y = 0.0, z = 0.0;   // lane < n: y and z of the candidate
    float x = 0.0f;            // lane < n: its coordinate
    bool drawn = false;        // z came from the state (not to be written back)
};

__device__ __forceinline__ AskOut ask_candidate(const RasterArgs& a, int b, int lane, float* s_M, char* scratch) {
    const int n = a.n;
    StateView S = state_view(a.state, n, a.lam);
    double* s_L = reinterpret_cast<double*>(scratch);              // [n][n]
    double* s_z = s_L + kMaxN * kMaxN;                              // [n + 3]
    float* s_X = reinterpret_cast<float*>(s_z + kMaxN + 3);         // [n]
    float* s_trig = s_X + kMaxN;                                     // [2][16]
    ChainK* s_ch = reinterpret_cast<ChainK*>(s_trig + 32);          // [kMaxArms]
    // the chains' parameters copied to LDS by one lane: the lanes below select
    // their arm's fields from LDS instead of holding both chains in scalar
    // registers through the whole prologue (which the kernel would spill)
    if (lane == 0) {
        s_ch[0] = a.fk.ch[0];
        s_ch[1] = a.fk.ch[1];
    }
    const int64_t gen64 = S.hdr->gen;
    const bool drawn = S.hdr->z_gen == gen64;
    const uint32_t gen = uint32_t(gen64);
    const uint64_t seed = S.hdr->seed;
    const uint32_t key0 = uint32_t(seed), key1 = uint32_t(seed >> 32);
    const int groups = (n + 3) / 4;
    // the state this lane needs after the draw, loaded first so that the
    // loads overlap the random-number arithmetic (the fences below would
    // otherwise hold them back)
    double mean_l = 0.0, off_l = 0.0, scale_l = 0.0, z_l = 0.0;
    if (lane < n) {
        mean_l = S.mean[lane];
        off_l = S.offset[lane];
        scale_l = S.scale[lane];
        z_l = S.Z[size_t(b) * n + lane];   // used when drawn
    }
    const double sigma = *S.sigma;
    for (int e = lane; e < n * n; e += kWave) s_L[e] = S.L[e];
    if (drawn) {
        if (lane < n) s_z[lane] = z_l;
    } else if (lane < 2 * groups) {
        draw_normal_pair(key0, key1, gen, b, lane >> 1, lane & 1, s_z + 2 * lane);
    }
    wave_sync();
    // the candidate's coordinates stay in registers until the end: a global
    // store issued here would make the forward kinematics below wait for it
    double y_l = 0.0, z_out = 0.0;
    float x_l = 0.0f;
    if (lane < n) {
        x_l = candidate_coord(s_L, s_z, n, lane, mean_l, sigma, off_l, scale_l, &y_l);
        z_out = s_z[lane];
        s_X[lane] = x_l;
    }
    wave_sync();
    // forward kinematics in three lane-parallel levels, so that the chain of
    // dependent trigonometric evaluations is two long instead of five; each
    // value comes from the same call with the same argument as in fk_pose and
    // fk_link, so the transforms carry the same bits as the FK kernel's.
    // s_trig per arm: sin, cos of alpha, beta, gamma [0..5], q1..q3 [6..8],
    // sin, cos of q1 [9, 10] and of the jaw angles phi+ [11, 12], phi- [13, 14].
    const int n_arms = a.fk.n_arms;
    {
        const int arm = lane >> 3, k = lane & 7;   // level 1: lane (arm, k), k < 6
        if (arm < n_arms && k < 6) {
            const float* th = s_X + 9 * arm;
            float* t = s_trig + 16 * arm;
            if (k < 3) {
                float sn, cs;
                sincosf(th[k], &sn, &cs);
                t[2 * k] = sn;
                t[2 * k + 1] = cs;
            } else {
                const int j = k - 3;
                t[6 + j] = decode_joint(th[6 + j], s_ch[arm].lb[j], s_ch[arm].ub[j]);
            }
        }
    }
    wave_sync();
    {
        const int arm = lane >> 3, k = lane & 7;   // level 2: q1 (k = 0), phi+ (k = 1), phi- (k = 2)
        if (arm < n_arms && k < 3) {
            float* t = s_trig + 16 * arm;
            float sn, cs;
            sincosf(k == 0 ? t[6] : fk_link_phi(k + 1, t + 6), &sn, &cs);
            t[9 + 2 * k] = sn;
            t[10 + 2 * k] = cs;
        }
    }
    wave_sync();
    // level 3: (arm, link) on lanes 0 .. 4 n_arms - 1, (arm, keypoint) on
    // lanes 8 .. 8 + 4 n_arms - 1
    const int arm = (lane & 7) >> 2, part = lane & 3;
    if ((lane < 8 && arm < n_arms) || (lane >= 8 && lane < 16 && arm < n_arms && a.kp)) {
        const ChainK& ch = s_ch[arm];
        const float* t = s_trig + 16 * arm;
        FkPose P;
        fk_pose_from(s_X + 9 * arm, t[0], t[1], t[2], t[3], t[4], t[5], t + 6, t[9], t[10], P);
        const int l = lane < 8 ? part : select4(part, ch.kp_link[0], ch.kp_link[1], ch.kp_link[2], ch.kp_link[3]);
        // sin, cos of fk_link_phi(l): phi+ for link 2, phi- for link 3, phi = 0 below (sin 0 = 0, cos 0 = 1)
        const float sp = l == 2 ? t[11] : l == 3 ? t[13] : 0.0f;
        const float cp = l == 2 ? t[12] : l == 3 ? t[14] : 1.0f;
        float M[12];
        fk_link_from(l, P, ch, sp, cp, M);
        if (lane < 8) {
#pragma unroll
            for (int e = 0; e < 12; e++) s_M[48 * arm + 12 * part + e] = M[e];
        } else {
            fk_keypoint(M, ch, part, a.fk.cam, a.kp + (size_t(b) * n_arms + arm) * 8 + 2 * part);
        }
    }
    AskOut o;
    o.y = y_l;
    o.z = z_out;
    o.x = x_l;
    o.drawn = drawn;
    return o;
}

// The candidate's global outputs (Z unless it was read, Y, X, the link
// transforms), written by wave 0 after the workgroup barrier that publishes
// s_M, so that the other waves do not wait while they are issued.
__device__ __forceinline__ void ask_store(const RasterArgs& a, int b, int lane, const float* s_M, const AskOut& o) {
    const int n = a.n;
    StateView S = state_view(a.state, n, a.lam);
    if (lane < n) {
        if (!o.drawn) S.Z[size_t(b) * n + lane] = o.z;
        S.Y[size_t(b) * n + lane] = o.y;
        a.X[size_t(b) * n + lane] = o.x;
    }
    const int n_arms = a.fk.n_arms;
    for (int e = lane; e < n_arms * 48; e += kWave) a.link_xf_out[size_t(b) * n_arms * 48 + e] = s_M[e];
}

// ---------------------------------------------------------------- triangle chunks

// Triangle chunks hold 64 triangles, one per lane, numbered over the meshes:
// chunks 0 .. C0 - 1 are mesh 0's, the next ones mesh 1's; C >= 1 chunks in
// all.  A chunk number past the last chunk stands for the last chunk, and a
// lane past its mesh's last triangle for that triangle: every load below is
// in bounds without a branch (a load in a branch makes the compiler wait for
// it at the branch's end), and `live` marks the lanes whose triangle counts.
struct ChunkLane {
    bool second;   // the chunk is mesh 1's
    int t;         // triangle of the lane in its mesh (clamped)
    bool live;
};

__device__ __forceinline__ ChunkLane chunk_lane(const MeshK& m0, const MeshK& m1, int C0, int C, int c, int lane) {
    const int cc = max(min(c, C - 1), 0);
    const bool second = cc >= C0;
    const int t = (cc - (second ? C0 : 0)) * kWave + lane;
    const int T = second ? m1.n_triangles : m0.n_triangles;
    return {second, min(t, T - 1), c < C && t < T};
}

// Vertex indices of lane `lane`'s triangle in chunk c.
__device__ __forceinline__ void load_chunk_indices(const MeshK& m0, const MeshK& m1, int C0, int C, int c, int lane,
                                                   int32_t* idx) {
    const ChunkLane cl = chunk_lane(m0, m1, C0, C, c, lane);
    const int32_t* tri = (cl.second ? m1.triangles : m0.triangles) + 3 * size_t(cl.t);
    idx[0] = tri[0];
    idx[1] = tri[1];
    idx[2] = tri[2];
}

// The three vertices of a lane's triangle: snapped points read from the
// workspace, or model-space positions and link-transform offsets to be
// projected when the chunk is rasterised.
template <bool FROM_SNAPPED>
struct ChunkVerts;
template <>
struct ChunkVerts<true> {
    int32_t X[3], Y[3];
    bool live;
    bool second;   // the triangle is mesh 1's
};
template <>
struct ChunkVerts<false> {
    float vx[3], vy[3], vz[3];
    int off[3];
    bool live;
};

// The vertices of lane `lane`'s triangle in chunk c, from the indices that
// load_chunk_indices read for the same chunk (valid vertex indices of the
// chunk's mesh in every lane).
template <bool FS>
__device__ __forceinline__ void gather_chunk(const RasterArgs& a, const MeshK& m0, const MeshK& m1, int C0, int C,
                                             int b, int c, int lane, const int32_t* idx, ChunkVerts<FS>& g) {
    const ChunkLane cl = chunk_lane(m0, m1, C0, C, c, lane);
    g.live = cl.live;
    if constexpr (FS) {
        g.second = cl.second;
        const int2* snap = reinterpret_cast<const int2*>(a.snapped) +
                           (size_t(b) * a.meshes.total_vertices + (cl.second ? m1.vertex_offset : m0.vertex_offset));
        for (int k = 0; k < 3; k++) {
            const int2 p = snap[idx[k]];
            g.X[k] = p.x;
            g.Y[k] = p.y;
        }
    } else {
        const float* V = cl.second ? m1.vertices : m0.vertices;
        const uint8_t* L = cl.second ? m1.vertex_link : m0.vertex_link;
        for (int k = 0; k < 3; k++) {
            const float* p = V + size_t(idx[k]) * 3;
            g.vx[k] = p[0];
            g.vy[k] = p[1];
            g.vz[k] = p[2];
            g.off[k] = (cl.second ? 48 : 0) + 12 * int(L[idx[k]]);
        }
    }
}

// Snapped points of a gathered chunk (INT32_MIN columns outside the meshes).
template <bool FS>
__device__ __forceinline__ void chunk_snapped(const ChunkVerts<FS>& g, const float* s_M, const CamK& cam, int32_t* X,
                                              int32_t* Y) {
    if constexpr (FS) {
        for (int k = 0; k < 3; k++) {
            X[k] = g.live ? g.X[k] : INT32_MIN;
            Y[k] = g.live ? g.Y[k] : 0;
        }
    } else {
        for (int k = 0; k < 3; k++) {
            X[k] = INT32_MIN;
            Y[k] = 0;
        }
        if (g.live)
            for (int k = 0; k < 3; k++) project_snap(s_M + g.off[k], g.vx[k], g.vy[k], g.vz[k], cam, X[k], Y[k]);
    }
}

// Where a workgroup's per-wave task queues live: `active` blocks of
// queue_bytes(NR) bytes from base, one per rasterising wave (waves past them
// help with the per-candidate phases only).
struct QueueLayout {
    char* base;
    int active;   // rasterising waves, 1 .. NT / 64
};

// One workgroup rasterises candidate b of the problem described by a into the
// image mask s_mask (LDS); NR narrow ring slots per wave (128, or 64 with
// drains before overflow).
template <bool FROM_SNAPPED, bool WRITE_MASK, bool COUNTS, int NT, int NR = kNarrowRing>
__device__ __forceinline__ void raster_body(const RasterArgs& a, const int b, unsigned long long* __restrict__ s_mask,
                                            const QueueLayout ql, const int tid) {
    constexpr int NW = NT / kWave;
    __shared__ float s_M[kMaxArms * 48];
    __shared__ int32_t s_red[2][NW];
    // [0] next chunk to claim; [1] bit m: a vertex of mesh m failed the near plane
    __shared__ int32_t s_ctl[2];

    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const int lx = lane & 7, ly = lane >> 3;
    const CamK& cam = a.cam;
    const int words = cam.words_x * cam.words_y;
    const int NA = ql.active;
    const QueueView Q = queue_view(ql.base + wave * queue_bytes(NR), NR);   // used by waves < NA only

    const int TV = a.meshes.total_vertices;
    const MeshK& m0 = a.meshes.m[0];
    const MeshK& m1 = a.meshes.m[1];
    const bool two = a.meshes.n_meshes > 1;
    const bool pretransform = FROM_SNAPPED && a.pretransform;
    // triangles in chunks of 64 (one per lane), numbered over the meshes
    const int C0 = (m0.n_triangles + kWave - 1) / kWave;
    const int C = two ? C0 + (m1.n_triangles + kWave - 1) / kWave : C0;
    // wave w starts with chunks w and 2 NA - 1 - w (the first chunk of one
    // wave pairs with the last of the first 2 NA, so that, when a mesh lists
    // its costly chunks first, the costliest pairs with the cheapest); it
    // claims each later chunk from an LDS counter two chunks ahead of the one
    // it rasterises (indices two ahead, vertex gathers one ahead), so all
    // waves finish within about one chunk of each other
    int c_cur = wave < NA ? wave : C, c_nxt = wave < NA ? 2 * NA - 1 - wave : C;
    if (tid == 0) {
        s_ctl[0] = 2 * NA;
        s_ctl[1] = 0;
    }

    AskOut ao;
    if (a.ask && NT > kWave) {
        // wave 0 starts on the candidate at once (its queues are not in use
        // yet); the other waves clear the mask
        if (wave == 0) ao = ask_candidate(a, b, lane, s_M, ql.base);
        else for (int w = tid - kWave; w < words; w += NT - kWave) s_mask[w] = 0ull;
    } else {
        for (int w = tid; w < words; w += NT) s_mask[w] = 0ull;
        if (a.ask) {
            if (wave == 0) ao = ask_candidate(a, b, lane, s_M, ql.base);
        } else if (!FROM_SNAPPED || a.pretransform) {
            for (int i = tid; i < a.meshes.n_meshes * 48; i += NT)
                s_M[i] = a.link_xf[size_t(b) * a.meshes.n_meshes * 48 + i];
        }
    }
    __syncthreads();
    if (a.ask && wave == 0) ask_store(a, b, lane, s_M, ao);
    // the vertex indices of the wave's first two chunks
    int32_t idx_cur[3], idx_nxt[3];   // read only for chunks < C
    if (C > 0) {   // no triangles at all: nothing to load
        load_chunk_indices(m0, m1, C0, C, c_cur, lane, idx_cur);
        load_chunk_indices(m0, m1, C0, C, c_nxt, lane, idx_nxt);
    }
    if (pretransform) {
        // transform, project and snap every vertex of this candidate once into the workspace
        int2* out = reinterpret_cast<int2*>(const_cast<int32_t*>(a.snapped)) + size_t(b) * TV;
        int culled = 0;   // bit m: one of this lane's vertices of mesh m failed the near plane
        // each lane's next vertex and link index are loaded (from a clamped,
        // valid index, with no branch) while it projects the current one
        struct VtxIn {
            float x, y, z;
            int off;      // the link transform in s_M: 48 floats per mesh, 12 per link
            bool second;
        };
        auto load_vtx = [&](int gv) {
            const int g = min(gv, TV - 1);
            VtxIn r;
            r.second = two && g >= m1.vertex_offset;
            const int v = g - (r.second ? m1.vertex_offset : m0.vertex_offset);
            const float* p = (r.second ? m1.vertices : m0.vertices) + size_t(v) * 3;
            r.x = p[0];
            r.y = p[1];
            r.z = p[2];
            r.off = (r.second ? 48 : 0) + 12 * int((r.second ? m1.vertex_link : m0.vertex_link)[v]);
            return r;
        };
        if (!two) {
            // one mesh: uniform bases, the vertex index is the lane's own
            const float* __restrict__ V = m0.vertices;
            const uint8_t* __restrict__ Lk = m0.vertex_link;
            for (int gv = tid; gv < TV; gv += NT) {
                int32_t X, Y;
                const bool ok = project_snap(s_M + 12 * int(Lk[gv]), V[3 * gv], V[3 * gv + 1], V[3 * gv + 2], cam,
                                             X, Y);
                culled |= ok ? 0 : 1;
                out[gv] = make_int2(X, Y);
            }
        } else {
            VtxIn cur = load_vtx(tid);
            for (int gv = tid; gv < TV; gv += NT) {
                const VtxIn nxt = load_vtx(gv + NT);
                int32_t X, Y;
                const bool ok = project_snap(s_M + cur.off, cur.x, cur.y, cur.z, cam, X, Y);
                culled |= ok ? 0 : (cur.second ? 2 : 1);
                out[gv] = make_int2(X, Y);
                cur = nxt;
            }
        }
        const unsigned long long c0 = __ballot(culled & 1), c1 = __ballot(culled & 2);
        if (lane == 0 && (c0 | c1)) atomicOr(&s_ctl[1], (c0 ? 1 : 0) | (c1 ? 2 : 0));
        __syncthreads();
    }
    // One-sided drawing: a closed mesh none of whose vertices failed the near
    // plane is rasterised from its triangles of positive signed area only --
    // the same pixel centres as all of its triangles (tk_mesh.closed).  Only
    // with the pre-transform is the near-plane test known before the set-up.
    const int near_culled = pretransform ? s_ctl[1] : 3;
    const bool one0 = m0.closed && !(near_culled & 1);
    const bool one1 = two && m1.closed && !(near_culled & 2);

    // queue state, the same in every lane of the wave: running slot counts
    // (head, tail) and task counts (queued, done) of the narrow and wide queues
    int n_head = 0, n_tail = 0, n_queued = 0, n_done = 0;
    int w_head = 0, w_tail = 0, w_queued = 0, w_done = 0;
    ChunkVerts<FROM_SNAPPED> g_cur;
    if (c_cur < C) gather_chunk(a, m0, m1, C0, C, b, c_cur, lane, idx_cur, g_cur);
    while (c_cur < C) {
        // the claim's result is read after the triangle setup below, which
        // covers its LDS round trip (this file is compiled without the
        // compiler's atomic optimizer, which would wait for it right here)
        int claim;   // read in lane 0 only
        if (lane == 0) claim = atomicAdd(&s_ctl[0], 1);
        ChunkVerts<FROM_SNAPPED> g_nxt;
        gather_chunk(a, m0, m1, C0, C, b, c_nxt, lane, idx_nxt, g_nxt);
        int c_new;
        {
            int32_t X[3], Y[3];
            chunk_snapped(g_cur, s_M, cam, X, Y);
            bool keep = g_cur.live;
            if constexpr (FROM_SNAPPED) {
                // back-facing (or degenerate) triangles of a one-sided mesh cover nothing new
                if (g_cur.second ? one1 : one0) {
                    const int64_t area2 = (int64_t(X[1]) - X[0]) * (int64_t(Y[2]) - Y[0]) -
                                          (int64_t(Y[1]) - Y[0]) * (int64_t(X[2]) - X[0]);
                    keep = keep && area2 > 0;
                }
            }
            // a chunk with nothing to draw (wholly back-facing in a plane-ordered
            // mesh) skips the set-up and queueing with one uniform branch
            const bool any = __ballot(keep) != 0ull;
            TriRec rec;
            bool valid = false;
            if (any) valid = keep && setup_triangle(X[0], Y[0], X[1], Y[1], X[2], Y[2], cam, rec);
            // claims exceed every chunk the wave holds (the counter starts at
            // 2 NA); the max keeps each wave's chunk numbers increasing regardless
            c_new = max(__builtin_amdgcn_readlane(claim, 0), c_nxt + 1);
            load_chunk_indices(m0, m1, C0, C, c_new, lane, idx_nxt);
            if (any) {
                const bool near = valid && (rec.flags & kNear);
                const bool narrow = near && is_narrow(rec.box_x);
                const bool wide = near && !narrow;
                // lane tasks: 8-column windows x 4-row bands (at most 8 x 15) for wide
                // boxes, kNarrowRows-row windows (at most 6) for narrow ones; both counts in one
                // wave scan, wide in the low and narrow in the high 16 bits
                const int cnt_w = wide ? task_windows(rec.box_x) * task_bands(rec.box_y) : 0;
                const int cnt_n = narrow ? narrow_tasks(rec.box_y) : 0;
                const int incl = wave_inclusive_sum(cnt_w | (cnt_n << 16));
                const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
                const unsigned long long nmask = __ballot(narrow), wmask = __ballot(wide);
                const int n_new = __popcll(nmask), w_new = __popcll(wmask);
                // a ring drains its pending tasks (fewer than 64) before it would overflow
                if (n_head - n_tail + n_new > Q.nmask + 1) {
                    run_round<true>(Q.na, Q.nb, Q.nstart, Q.mark, Q.nmask, n_tail, n_head, n_done, n_queued - n_done,
                                    lane, s_mask, cam.words_x);
                    n_done = n_queued;
                    n_tail = n_head;
                }
                if (w_head - w_tail + w_new > kWideRing) {
                    run_round<false>(Q.wa, Q.wb, Q.wstart, Q.mark, kWideRing - 1, w_tail, w_head, w_done,
                                     w_queued - w_done, lane, s_mask, cam.words_x);
                    w_done = w_queued;
                    w_tail = w_head;
                }
                if (narrow || wide) {
                    const NearRec r = pack_near(rec);
                    const unsigned long long m = narrow ? nmask : wmask;
                    const int rank = int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
                    if (narrow) {
                        const int slot = (n_head + rank) & Q.nmask;
                        Q.na[slot] = r.a;
                        Q.nb[slot] = r.b;
                        Q.nstart[slot] = n_queued + (incl >> 16) - cnt_n;
                    } else {
                        const int slot = (w_head + rank) & (kWideRing - 1);
                        Q.wa[slot] = r.a;
                        Q.wb[slot] = r.b;
                        Q.wstart[slot] = w_queued + (incl & 0xffff) - cnt_w;
                    }
                }
                n_head += n_new;
                n_queued += total >> 16;
                w_head += w_new;
                w_queued += total & 0xffff;
                wave_sync();   // queued records written by other lanes are read below
                while (n_queued - n_done >= kWave) {
                    n_tail = run_round<true>(Q.na, Q.nb, Q.nstart, Q.mark, Q.nmask, n_tail, n_head, n_done, kWave, lane,
                                             s_mask, cam.words_x);
                    n_done += kWave;
                }
                while (w_queued - w_done >= kWave) {
                    w_tail = run_round<false>(Q.wa, Q.wb, Q.wstart, Q.mark, kWideRing - 1, w_tail, w_head, w_done, kWave,
                                              lane, s_mask, cam.words_x);
                    w_done += kWave;
                }
                // triangles needing 64-bit edge functions or big boxes: the whole wave
                // on one triangle at a time, its record broadcast from its lane
                unsigned long long todo = __ballot(valid && !near);
                while (todo) {
                    const int j = __builtin_ctzll(todo);
                    todo &= todo - 1;
                    TriRec br;
#pragma unroll
                    for (int e = 0; e < 3; e++) {
                        br.e0lo[e] = __builtin_amdgcn_readlane(rec.e0lo[e], j);
                        br.e0hi[e] = __builtin_amdgcn_readlane(rec.e0hi[e], j);
                        br.dx[e] = __builtin_amdgcn_readlane(rec.dx[e], j);
                        br.dy[e] = __builtin_amdgcn_readlane(rec.dy[e], j);
                    }
                    br.box_x = __builtin_amdgcn_readlane(rec.box_x, j);
                    br.box_y = __builtin_amdgcn_readlane(rec.box_y, j);
                    br.flags = __builtin_amdgcn_readlane(rec.flags, j);
                    br.pad = 0;
                    cover_big(br, lx, ly, lane, s_mask, cam.words_x);
                }
            }
        }
        g_cur = g_nxt;
        c_cur = c_nxt;
        c_nxt = c_new;
    }
    // the last partial rounds
    if (n_queued > n_done)
        run_round<true>(Q.na, Q.nb, Q.nstart, Q.mark, Q.nmask, n_tail, n_head, n_done, n_queued - n_done, lane, s_mask,
                        cam.words_x);
    if (w_queued > w_done)
        run_round<false>(Q.wa, Q.wb, Q.wstart, Q.mark, kWideRing - 1, w_tail, w_head, w_done, w_queued - w_done, lane,
                         s_mask, cam.words_x);
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


template <bool FROM_SNAPPED, bool WRITE_MASK, bool COUNTS, int NT>
__global__ __launch_bounds__(NT) void raster_kernel(RasterArgs a) {
    extern __shared__ unsigned long long s_dyn[];
    __shared__ WaveQueues s_queue[NT / kWave];
    raster_body<FROM_SNAPPED, WRITE_MASK, COUNTS, NT>(
        a, blockIdx.x, s_dyn, QueueLayout{reinterpret_cast<char*>(s_queue), NT / kWave}, threadIdx.x);
}

// Many problems in one launch: workgroups first[i] .. first[i + 1] - 1 draw
// and rasterise the candidates of problem prob[i] (table entries in device
// memory, read through a uniform pointer).
struct BatchLaunch {
    const RasterArgs* table;
    int32_t count;
    int32_t prob[kMaxBatch];
    int32_t first[kMaxBatch + 1];
};

template <int NT>
__global__ __launch_bounds__(NT) void raster_batch_kernel(BatchLaunch L) {
    const int g = blockIdx.x;
    int lo = 0;   // last i with first[i] <= g
    for (int step = kMaxBatch / 2; step > 0; step >>= 1)
        if (lo + step < L.count && L.first[lo + step] <= g) lo += step;
    const RasterArgs& a = L.table[L.prob[lo]];
    extern __shared__ unsigned long long s_dyn[];
    __shared__ WaveQueues s_queue[NT / kWave];
    raster_body<true, false, true, NT>(a, g - L.first[lo], s_dyn,
                                       QueueLayout{reinterpret_cast<char*>(s_queue), NT / kWave}, threadIdx.x);
}

// Persistent form: a grid of resident workgroups, each claiming (problem,
// candidate) items from a device counter until all are taken.  Problem
// prob[i] owns items first[i] .. first[i + 1] - 1, one per candidate; the host
// lists the problems costliest per candidate first, so the last claims are
// cheap (longest-first list scheduling over the whole batch).  Every item uses
// the same 1024-thread workgroup with its own LDS layout: the image mask, then
// NR narrow ring slots per wave for active[i] rasterising waves.  counter[0] is the next item and counter[1] the workgroups that have
// finished; the last to finish resets both, so consecutive launches (and graph
// replays) need no clearing.
struct PersistLaunch {
    const RasterArgs* table;
    int32_t* counter;
    int32_t count;
    int32_t prob[kMaxBatch];
    int32_t first[kMaxBatch + 1];
    int32_t active[kMaxBatch];
};

template <int NT, int NR>
__global__ __launch_bounds__(NT) void raster_persistent_kernel(PersistLaunch L) {
    extern __shared__ unsigned long long s_dyn[];
    __shared__ int32_t s_item;
    const int total = L.first[L.count];
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&L.counter[0], 1);
        __syncthreads();
        const int item = s_item;
        __syncthreads();   // every thread has read the claim before the next one overwrites it
        if (item >= total) break;
        int lo = 0;   // last i with first[i] <= item
        for (int step = kMaxBatch / 2; step > 0; step >>= 1)
            if (lo + step < L.count && L.first[lo + step] <= item) lo += step;
        const RasterArgs& a = L.table[L.prob[lo]];
        const size_t mask_bytes = (size_t(a.cam.words_x) * a.cam.words_y * 8 + 15) & ~size_t(15);
        // the thread index passes through an empty asm statement each item, so
        // that nothing derived from it is hoisted out of the loop and held in
        // registers across the whole body
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        raster_body<true, false, true, NT, NR>(a, item - L.first[lo], s_dyn,
                                               QueueLayout{reinterpret_cast<char*>(s_dyn) + mask_bytes, L.active[lo]},
                                               tid);
        __syncthreads();   // the item's last LDS reads are done before the next item clears the mask
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&L.counter[1], 1) == int(gridDim.x) - 1) {
            L.counter[0] = 0;
            L.counter[1] = 0;
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
    const MeshK mesh = mi == 0 ? a.meshes.m[0] : a.meshes.m[1];   // selected, not indexed: no private copy of the arguments
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
    __shared__ int s_culled;   // bit m: a vertex of mesh m fails the near plane
    if (threadIdx.x < 4) s_acc[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) s_culled = 0;
    __syncthreads();
    for (int mi = 0; mi < a.meshes.n_meshes; mi++) {
        const MeshK mesh = mi == 0 ? a.meshes.m[0] : a.meshes.m[1];
        const float* M = a.link_xf + (size_t(b) * a.meshes.n_meshes + mi) * 48;
        bool any = false;
        for (int v = threadIdx.x; v < mesh.n_vertices; v += blockDim.x) {
            const float* p = mesh.vertices + size_t(v) * 3;
            int32_t X, Y;
            any |= !project_snap(M + 12 * mesh.vertex_link[v], p[0], p[1], p[2], a.cam, X, Y);
        }
        if (any) atomicOr(&s_culled, 1 << mi);
    }
    __syncthreads();
    unsigned long long kept = 0, pix = 0, pairs = 0, huge = 0;
    for (int mi = 0; mi < a.meshes.n_meshes; mi++) {
        const MeshK mesh = mi == 0 ? a.meshes.m[0] : a.meshes.m[1];   // selected, not indexed: no private copy of the arguments
        const float* M = a.link_xf + (size_t(b) * a.meshes.n_meshes + mi) * 48;
        // the triangles the one-sided path of the workspace forms draws
        const bool one = mesh.closed && !((s_culled >> mi) & 1);
        for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < mesh.n_triangles; t += gridDim.x * blockDim.x) {
            int32_t X[3], Y[3];
            for (int k = 0; k < 3; k++) {
                const int32_t v = mesh.triangles[3 * t + k];
                const float* p = mesh.vertices + size_t(v) * 3;
                project_snap(M + 12 * mesh.vertex_link[v], p[0], p[1], p[2], a.cam, X[k], Y[k]);
            }
            if (one && (int64_t(X[1]) - X[0]) * (int64_t(Y[2]) - Y[0]) - (int64_t(Y[1]) - Y[0]) * (int64_t(X[2]) - X[0]) <= 0)
                continue;
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
    // queues, transforms, count partials and the chunk counter (padded to 8
    // bytes: the 64-bit words of the dynamic mask follow)
    return sizeof(WaveQueues) * (NT / kWave) + sizeof(float) * kMaxArms * 48 + sizeof(int32_t) * 2 * (NT / kWave) +
           sizeof(int64_t);
}

template <bool FS, bool WM, bool CN, int NT>
tk_status launch_raster_nt(const RasterArgs& a, size_t lds, hipStream_t s, const char* what) {
    auto kern = raster_kernel<FS, WM, CN, NT>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    static size_t static_bytes = 0;
    std::call_once(once, [&] {
        // the LDS budget of the image mask assumes the kernel's static LDS is at most static_lds<NT>()
        hipFuncAttributes fa{};
        attr_err = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern));
        static_bytes = fa.sharedSizeBytes;
        if (attr_err == hipSuccess)
            attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           int(kLdsLimit - static_lds<NT>()));
    });
    if (attr_err != hipSuccess)
        return fail(TK_ERR_DEVICE, "%s: cannot raise the dynamic LDS limit: %s", what, hipGetErrorString(attr_err));
    if (static_bytes > static_lds<NT>())
        return fail(TK_ERR_DEVICE, "%s: kernel has %zu bytes of static LDS, the launch assumes at most %zu", what,
                    static_bytes, static_lds<NT>());
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
    a->ask = 0;
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

// Arguments of the ask-eval launch (workspace not yet attached).
tk_status ask_eval_args(void* d_state, int32_t n, int32_t lambda, const tk_chain* chains, int32_t n_arms,
                        const tk_mesh* meshes, const tk_camera* cam, const uint64_t* d_target, float* d_X,
                        float* d_link_xf, float* d_kp, int32_t* d_counts, RasterArgs* a) {
    TK_REQUIRE(d_state != nullptr && (reinterpret_cast<uintptr_t>(d_state) & 255) == 0,
               "state must be a 256-byte aligned device pointer");
    TK_REQUIRE(lambda >= 2 && lambda <= kMaxLambda, "lambda = %d outside 2..%d", lambda, kMaxLambda);
    TK_REQUIRE(n_arms >= 1 && n_arms <= kMaxArms && n == 9 * n_arms, "n = %d must be 9 x n_arms (n_arms = %d)", n,
               n_arms);
    if (tk_status st = common_raster_checks(lambda, meshes, n_arms, cam, a)) return st;
    TK_REQUIRE(d_X && d_link_xf && d_target && d_counts, "X / link_xf / target / counts is NULL");
    if (tk_status st = make_fk_args(chains, n_arms, cam, &a->fk)) return st;
    a->fk.batch = lambda;
    a->ask = 1;
    a->n = n;
    a->lam = lambda;
    a->state = d_state;
    a->X = d_X;
    a->link_xf_out = d_link_xf;
    a->kp = d_kp;
    a->target = reinterpret_cast<const unsigned long long*>(d_target);
    a->counts = d_counts;
    return TK_OK;
}

// ---------------------------------------------------------------- static scratch of the allocation-free entry point

// The snapped-vertex workspace of tk_cmaes_ask_eval_noalloc: one array per
// device, allocated when the code object is loaded and held until the process
// ends.  Host code never uses this name as an address (on the host it is a
// stand-in symbol); it uses the device address that hipGetSymbolAddress
// returns, queried once per device with that device current.
static __device__ __align__(256) unsigned char scratch[TK_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (queried on the first
// call on that device).
tk_status noalloc_scratch(void** out, const char* what) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(TK_ERR_DEVICE, "%s: hipGetDevice: %s", what, hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(TK_ERR_UNSUPPORTED, "%s: device %d beyond %d", what, dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(TK_ERR_DEVICE, "%s: hipGetSymbolAddress of the static scratch on device %d: %s", what, dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TK_OK;
}

}  // namespace

size_t batch_raster_entry_bytes() { return sizeof(RasterArgs); }

tk_status batch_describe_raster(const tk_problem& p, void* dst) {
    TK_REQUIRE(p.d_state != nullptr && (reinterpret_cast<uintptr_t>(p.d_state) & 255) == 0,
               "state must be a 256-byte aligned device pointer");
    TK_REQUIRE(p.lambda >= 2 && p.lambda <= kMaxLambda, "lambda = %d outside 2..%d", p.lambda, kMaxLambda);
    TK_REQUIRE(p.n_arms >= 1 && p.n_arms <= kMaxArms && p.n == 9 * p.n_arms, "n = %d must be 9 x n_arms (n_arms = %d)",
               p.n, p.n_arms);
    RasterArgs a;
    std::memset(&a, 0, sizeof a);
    if (tk_status st = common_raster_checks(p.lambda, p.meshes, p.n_arms, &p.cam, &a)) return st;
    TK_REQUIRE(p.d_X && p.d_link_xf && p.d_target && p.d_counts, "X / link_xf / target / counts is NULL");
    TK_REQUIRE(p.d_ws != nullptr, "batched problems need a workspace (tk_raster_workspace_bytes)");
    TK_REQUIRE(p.threads == 0 || p.threads == 256 || p.threads == 512 || p.threads == 1024,
               "threads = %d must be 0, 256, 512 or 1024", p.threads);
    if (p.threads) {
        const size_t need = mask_lds_bytes(a.cam) + (p.threads == 1024   ? static_lds<1024>()
                                                     : p.threads == 512 ? static_lds<512>()
                                                                        : static_lds<256>());
        if (need > kLdsLimit)
            return fail(TK_ERR_UNSUPPORTED, "%d threads need %zu bytes of LDS at %dx%d (limit %zu)", p.threads, need,
                        p.cam.width, p.cam.height, kLdsLimit);
    }
    if (tk_status st = make_fk_args(p.chains, p.n_arms, &p.cam, &a.fk)) return st;
    a.fk.batch = p.lambda;
    a.ask = 1;
    a.n = p.n;
    a.lam = p.lambda;
    a.state = p.d_state;
    a.X = p.d_X;
    a.link_xf_out = p.d_link_xf;
    a.kp = p.d_kp;
    a.target = reinterpret_cast<const unsigned long long*>(p.d_target);
    a.counts = p.d_counts;
    if (tk_status st = attach_workspace(&a, p.d_ws, p.ws_bytes, "tk_batch_describe")) return st;
    std::memcpy(dst, &a, sizeof a);
    return TK_OK;
}

namespace {

// threads of problem p's workgroups: its choice, else the widest that fits
int batch_threads(const tk_problem& p) {
    if (p.threads) return p.threads;
    const size_t lds = mask_lds_bytes(make_cam(p.cam));
    if (lds + static_lds<1024>() <= kLdsLimit) return 1024;
    if (lds + static_lds<512>() <= kLdsLimit) return 512;
    return 256;
}

template <int NT>
tk_status launch_raster_batch(const BatchLaunch& L, size_t lds, hipStream_t s) {
    auto kern = raster_batch_kernel<NT>;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(kLdsLimit - static_lds<NT>()));
    });
    if (attr_err != hipSuccess)
        return fail(TK_ERR_DEVICE, "tk_batch_ask_eval: cannot raise the dynamic LDS limit: %s",
                    hipGetErrorString(attr_err));
    hipLaunchKernelGGL(kern, dim3(L.first[L.count]), dim3(NT), lds, s, L);
    return check_launch("tk_batch_ask_eval");
}

constexpr int kPersistThreads = 1024;
// static LDS of the persistent kernel: transforms, count partials, control words, the claimed item
constexpr size_t kPersistStatic = sizeof(float) * kMaxArms * 48 + sizeof(int32_t) * 2 * (kPersistThreads / kWave) +
                                  sizeof(int64_t) + 16;
constexpr size_t kPersistDynamic = kLdsLimit - kPersistStatic;

}  // namespace

// Rasterising waves of a problem's workgroup in the persistent kernel with nr
// narrow ring slots per wave: as many as fit beside the image mask, at most 16.
int persist_active(const CamK& cam, int nr) {
    const size_t mask = (mask_lds_bytes(cam) + 15) & ~size_t(15);
    if (mask >= kPersistDynamic) return 0;
    return int(std::min<size_t>(kPersistThreads / kWave, (kPersistDynamic - mask) / queue_bytes(nr)));
}

template <int NR>
tk_status launch_persistent(const PersistLaunch& L, int cus, hipStream_t s) {
    auto kern = raster_persistent_kernel<kPersistThreads, NR>;
    static std::once_flag once;
    static hipError_t err = hipSuccess;
    static size_t static_bytes = 0;
    std::call_once(once, [&] {
        hipFuncAttributes fa{};
        err = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kern));
        static_bytes = fa.sharedSizeBytes;
        if (err == hipSuccess)
            err = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                      int(kPersistDynamic));
    });
    if (err != hipSuccess)
        return fail(TK_ERR_DEVICE, "tk_batch_ask_eval_persistent: kernel set-up: %s", hipGetErrorString(err));
    if (static_bytes > kPersistStatic)
        return fail(TK_ERR_DEVICE, "tk_batch_ask_eval_persistent: kernel has %zu bytes of static LDS, %zu assumed",
                    static_bytes, kPersistStatic);
    hipLaunchKernelGGL(kern, dim3(cus), dim3(kPersistThreads), kPersistDynamic, s, L);
    return check_launch("tk_batch_ask_eval_persistent");
}

// All problems in one persistent launch per kMaxBatch problems, costliest
// per candidate first (image pixels times the square root of the triangle
// count as the estimate); 128 narrow ring slots when every image of the
// launch leaves room for 16 such waves, else 64.  counters: device int32
// pairs, one per launch.
tk_status batch_launch_persistent(const tk_problem* problems, int32_t n, const void* d_entries, int32_t* d_counters,
                                  hipStream_t s) {
    static std::once_flag once;
    static hipError_t dev_err = hipSuccess;
    static int cus = 0;
    std::call_once(once, [&] {
        int dev = 0;
        dev_err = hipGetDevice(&dev);
        if (dev_err == hipSuccess) dev_err = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    });
    if (dev_err != hipSuccess || cus < 1)
        return fail(TK_ERR_DEVICE, "tk_batch_ask_eval_persistent: device query: %s", hipGetErrorString(dev_err));
    std::vector<int> order(n);
    std::vector<double> cost(n);
    for (int i = 0; i < n; i++) {
        const tk_problem& p = problems[i];
        int64_t tris = 0;
        for (int m = 0; m < p.n_arms; m++) tris += p.meshes[m].n_triangles;
        cost[i] = double(p.cam.width) * p.cam.height * std::sqrt(double(tris) + 1000.0);
        order[i] = i;
        if (persist_active(make_cam(p.cam), 64) == 0)
            return fail(TK_ERR_UNSUPPORTED, "tk_batch_ask_eval_persistent: problem %d: image %dx%d leaves no LDS for "
                        "the task queues", i, p.cam.width, p.cam.height);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    for (int base = 0, launch = 0; base < n; base += kMaxBatch, launch++) {
        PersistLaunch L;
        std::memset(&L, 0, sizeof L);
        L.table = static_cast<const RasterArgs*>(d_entries);
        L.counter = d_counters + 2 * launch;
        L.count = std::min(kMaxBatch, n - base);
        bool wide_rings = true;
        for (int i = 0; i < L.count; i++)
            wide_rings &= persist_active(make_cam(problems[order[base + i]].cam), kNarrowRing) == kPersistThreads / kWave;
        for (int i = 0; i < L.count; i++) {
            const tk_problem& p = problems[order[base + i]];
            L.prob[i] = order[base + i];
            L.first[i + 1] = L.first[i] + p.lambda;
            L.active[i] = persist_active(make_cam(p.cam), wide_rings ? kNarrowRing : 64);
        }
        if (tk_status st = wide_rings ? launch_persistent<kNarrowRing>(L, cus, s) : launch_persistent<64>(L, cus, s))
            return st;
    }
    return TK_OK;
}

// Problems grouped by workgroup size; one launch per group of at most kMaxBatch.
tk_status batch_launch_raster(const tk_problem* problems, int32_t n, const void* d_entries, hipStream_t s) {
    const int sizes[3] = {1024, 512, 256};
    for (int nt : sizes) {
        BatchLaunch L;
        std::memset(&L, 0, sizeof L);
        L.table = static_cast<const RasterArgs*>(d_entries);
        size_t lds = 0;
        auto flush = [&]() -> tk_status {
            if (L.count == 0) return TK_OK;
            tk_status st = nt == 1024 ? launch_raster_batch<1024>(L, lds, s)
                         : nt == 512  ? launch_raster_batch<512>(L, lds, s)
                                      : launch_raster_batch<256>(L, lds, s);
            L.count = 0;
            L.first[0] = 0;
            lds = 0;
            return st;
        };
        for (int i = 0; i < n; i++) {
            if (batch_threads(problems[i]) != nt) continue;
            L.prob[L.count] = i;
            L.first[L.count + 1] = L.first[L.count] + problems[i].lambda;
            L.count++;
            lds = std::max(lds, mask_lds_bytes(make_cam(problems[i].cam)));
            if (L.count == kMaxBatch)
                if (tk_status st = flush()) return st;
        }
        if (tk_status st = flush()) return st;
    }
    return TK_OK;
}

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

tk_status tk_cmaes_ask_eval(void* d_state, int32_t n, int32_t lambda, const tk_chain* chains, int32_t n_arms,
                            const tk_mesh* meshes, const tk_camera* cam, const uint64_t* d_target, float* d_X,
                            float* d_link_xf, float* d_kp, int32_t* d_counts, void* d_ws, size_t ws_bytes,
                            tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = ask_eval_args(d_state, n, lambda, chains, n_arms, meshes, cam, d_target, d_X, d_link_xf, d_kp,
                                     d_counts, &a))
        return st;
    if (tk_status st = attach_workspace(&a, d_ws, ws_bytes, "tk_cmaes_ask_eval")) return st;
    if (a.pretransform)
        return launch_raster<true, false, true>(a, reinterpret_cast<hipStream_t>(s), "tk_cmaes_ask_eval");
    return launch_raster<false, false, true>(a, reinterpret_cast<hipStream_t>(s), "tk_cmaes_ask_eval");
}

tk_status tk_cmaes_ask_eval_noalloc(void* d_state, int32_t n, int32_t lambda, const tk_chain* chains,
                                    int32_t n_arms, const tk_mesh* meshes, const tk_camera* cam,
                                    const uint64_t* d_target, float* d_X, float* d_link_xf, float* d_kp,
                                    int32_t* d_counts, tk_stream s) {
    clear_error();
    RasterArgs a;
    if (tk_status st = ask_eval_args(d_state, n, lambda, chains, n_arms, meshes, cam, d_target, d_X, d_link_xf, d_kp,
                                     d_counts, &a))
        return st;
    const size_t need = tk_raster_workspace_bytes(lambda, meshes, n_arms);
    if (need > TK_NOALLOC_SCRATCH_BYTES)
        return fail(TK_ERR_UNSUPPORTED,
                    "tk_cmaes_ask_eval_noalloc: %d candidates x %d vertices need %zu bytes of scratch, the "
                    "library's static scratch holds %zu (use tk_cmaes_ask_eval with a workspace)",
                    lambda, a.meshes.total_vertices, need, size_t(TK_NOALLOC_SCRATCH_BYTES));
    void* ws = nullptr;
    if (tk_status st = noalloc_scratch(&ws, "tk_cmaes_ask_eval_noalloc")) return st;
    if (tk_status st = attach_workspace(&a, ws, TK_NOALLOC_SCRATCH_BYTES, "tk_cmaes_ask_eval_noalloc")) return st;
    return launch_raster<true, false, true>(a, reinterpret_cast<hipStream_t>(s), "tk_cmaes_ask_eval_noalloc");
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
