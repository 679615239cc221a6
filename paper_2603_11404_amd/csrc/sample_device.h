// Device functions of CMA-ES sampling shared by the sample kernel, the fused
// tell-ask kernel and the ask-eval raster kernel, so that every path draws
// identical candidates.  Random numbers: Philox4x32-10 (Salmon et al., SC'11)
// keyed by the seed with counter (group j, candidate k, generation g, 0),
// mapped to normals by Box-Muller in FP64.
#pragma once

#include "tk_internal.h"

namespace tk {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- Philox4x32-10

struct U4 { uint32_t x, y, z, w; };

__device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = uint64_t(0xD2511F53u) * c.x;
        uint64_t p1 = uint64_t(0xCD9E8D57u) * c.z;
        U4 o;
        o.x = uint32_t(p1 >> 32) ^ c.y ^ k0;
        o.y = uint32_t(p1);
        o.z = uint32_t(p0 >> 32) ^ c.w ^ k1;
        o.w = uint32_t(p0);
        c = o;
    }
    return c;
}

// Box-Muller: radius sqrt(-2 ln u1) and angle 2 pi u2 from two 32-bit words
// mapped to the open interval (0, 1).  The angle is taken in half turns,
// 2 u2 (exact), through sincospi: the cosine and sine of 2 pi u2 without
// rounding that product, and with a trivial argument reduction.
__device__ inline double bm_radius(uint32_t a) {
    const double u1 = (double(a) + 0.5) * 0x1p-32;
    return sqrt(-2.0 * log(u1));
}

__device__ inline double bm_half_turns(uint32_t b) {
    const double u2 = (double(b) + 0.5) * 0x1p-32;
    return 2.0 * u2;
}

__device__ inline void box_muller(uint32_t a, uint32_t b, double* z0, double* z1) {
    const double r = bm_radius(a);
    double s, c;
    sincospi(bm_half_turns(b), &s, &c);
    *z0 = r * c;
    *z1 = r * s;
}

// Normals 4j + 2h, 4j + 2h + 1 (h = 0, 1) of candidate k in generation g:
// Philox block (j, k, g, 0), its h-th Box-Muller pair.
__device__ inline void draw_normal_pair(uint32_t key0, uint32_t key1, uint32_t g, int k, int j, int h, double z[2]) {
    const U4 r = philox4x32_10(U4{uint32_t(j), uint32_t(k), g, 0u}, key0, key1);
    if (h == 0)
        box_muller(r.x, r.y, &z[0], &z[1]);
    else
        box_muller(r.z, r.w, &z[0], &z[1]);
}

// Normals 4j .. 4j + 3 of candidate k in generation g: one Philox block with
// counter (j, k, g, 0), two Box-Muller pairs.
__device__ inline void draw_normals(uint32_t key0, uint32_t key1, uint32_t g, int k, int j, double z[4]) {
    const U4 r = philox4x32_10(U4{uint32_t(j), uint32_t(k), g, 0u}, key0, key1);
    box_muller(r.x, r.y, &z[0], &z[1]);
    box_muller(r.z, r.w, &z[2], &z[3]);
}

// The first `count` (1 ... 4) of those normals, each with exactly the
// arithmetic of box_muller; the others are not computed.
__device__ inline void draw_normals_first(uint32_t key0, uint32_t key1, uint32_t g, int k, int j, int count,
                                          double z[4]) {
    const U4 r = philox4x32_10(U4{uint32_t(j), uint32_t(k), g, 0u}, key0, key1);
    const uint32_t a[2] = {r.x, r.z}, b[2] = {r.y, r.w};
#pragma unroll
    for (int h = 0; h < 2; h++) {
        if (2 * h < count) {
            const double rad = bm_radius(a[h]);
            double sn, cs;
            sincospi(bm_half_turns(b[h]), &sn, &cs);   // the same call as box_muller: the same bits
            z[2 * h] = rad * cs;
            if (2 * h + 1 < count) z[2 * h + 1] = rad * sn;
        }
    }
}

// y_i = sum_j L_ij z_j (L: a square root of C, n x n row-major), x_i = m_i +
// sigma y_i, theta_i = offset_i + scale_i x_i (FP32)
__device__ inline float candidate_coord(const double* L, const double* z, int n, int i, double mean_i, double sigma,
                                        double offset_i, double scale_i, double* y_out) {
    double y = 0.0;
    for (int j = 0; j < n; j++) y += L[i * n + j] * z[j];
    *y_out = y;
    const double x = mean_i + sigma * y;
    return float(offset_i + scale_i * x);
}

}  // namespace tk
