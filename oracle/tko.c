/*
 * tko.c -- plain CPU oracle (test infrastructure only; see tko.h).
 *
 * Every function is the definition written out, in FP64 for geometry and
 * int64 for the raster.  Nothing here is blocked, fused or reordered beyond
 * restricting each triangle's pixel loop to its bounding box.
 */
#include "tko.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TKO_PI 3.14159265358979323846
#define TKO_GUARD 32768.0 /* guard band in pixels */

/* ---- Sec. III-A.3: cosine reparameterisation of the joint limits ---- */
double tko_decode(double qhat, double lb, double ub) {
    return lb + (ub - lb) / 2.0 * (1.0 - cos(TKO_PI * (qhat - lb) / (ub - lb)));
}

double tko_encode(double q, double lb, double ub) {
    return lb + (ub - lb) / TKO_PI * acos(1.0 - 2.0 * (q - lb) / (ub - lb));
}

/* ---- elementary rotations (right-handed, active) ---- */
static void rot_x(double a, double R[9]) {
    double c = cos(a), s = sin(a);
    double r[9] = {1, 0, 0, 0, c, -s, 0, s, c};
    memcpy(R, r, sizeof r);
}
static void rot_y(double a, double R[9]) {
    double c = cos(a), s = sin(a);
    double r[9] = {c, 0, s, 0, 1, 0, -s, 0, c};
    memcpy(R, r, sizeof r);
}
static void rot_z(double a, double R[9]) {
    double c = cos(a), s = sin(a);
    double r[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
    memcpy(R, r, sizeof r);
}
static void mat3_mul(const double A[9], const double B[9], double C[9]) {
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(C, t, sizeof t);
}
/* 3x4 affine compose: C = A * B (both [R|t]) */
static void aff_mul(const double A[12], const double B[12], double C[12]) {
    double t[12];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 4; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[4 * i + k] * B[4 * k + j];
            if (j == 3) s += A[4 * i + 3];
            t[4 * i + j] = s;
        }
    }
    memcpy(C, t, sizeof t);
}
static void aff_from_rot(const double R[9], double x, double y, double z, double T[12]) {
    for (int i = 0; i < 3; i++) {
        T[4 * i + 0] = R[3 * i + 0];
        T[4 * i + 1] = R[3 * i + 1];
        T[4 * i + 2] = R[3 * i + 2];
    }
    T[3] = x; T[7] = y; T[11] = z;
}

/* ---- Sec. III-A.3: look-at pose ---- */
void tko_pose(double alpha, double beta, double gamma, double x, double y, double z, double T[12]) {
    double Rx[9], Ry[9], Rz[9], R[9];
    rot_x(alpha, Rx); rot_y(gamma, Ry); rot_z(beta, Rz);
    mat3_mul(Ry, Rx, R);
    mat3_mul(R, Rz, R);
    aff_from_rot(R, x, y, z, T);
}

/* ---- link chain of the procedural instrument (robot frame = wrist pitch) ---- */
void tko_chain_links(const double q[3], const tko_chain* ch, double T[4][12]) {
    static const double I[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    double R[9], pitch[12], yaw_origin[12], tmp[12];
    memcpy(T[0], I, sizeof I);                      /* shaft */
    rot_x(q[0], R);
    aff_from_rot(R, 0, 0, 0, pitch);
    memcpy(T[1], pitch, sizeof pitch);              /* wrist: Rx(q1) */
    double Itr[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, ch->d_pitch_yaw};
    aff_mul(pitch, Itr, yaw_origin);                /* Rx(q1) Tr(0,0,d) */
    for (int side = 0; side < 2; side++) {
        double phi = side == 0 ? q[1] + 0.5 * q[2] : q[1] - 0.5 * q[2];
        rot_y(phi, R);
        aff_from_rot(R, 0, 0, 0, tmp);
        aff_mul(yaw_origin, tmp, T[2 + side]);      /* ... Ry(q2 +- q3/2) */
    }
}

void tko_fk(const double theta[9], const tko_chain* ch, double M[4][12]) {
    double Trc[12], L[4][12], q[3];
    tko_pose(theta[0], theta[1], theta[2], theta[3], theta[4], theta[5], Trc);
    for (int j = 0; j < 3; j++) q[j] = tko_decode(theta[6 + j], ch->q_lb[j], ch->q_ub[j]);
    tko_chain_links(q, ch, L);
    for (int l = 0; l < 4; l++) aff_mul(Trc, L[l], M[l]);
}

/* ---- transform, pinhole projection, Q8 snap ---- */
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

void tko_project_snap(const double M[4][12], const float* vertices, const uint8_t* vlink, int32_t V,
                      const tko_camera* cam, double* uv, int32_t* snapped, uint8_t* flags) {
    for (int32_t i = 0; i < V; i++) {
        const double* m = M[vlink[i]];
        double vx = vertices[3 * i], vy = vertices[3 * i + 1], vz = vertices[3 * i + 2];
        double X = m[0] * vx + m[1] * vy + m[2] * vz + m[3];
        double Y = m[4] * vx + m[5] * vy + m[6] * vz + m[7];
        double Z = m[8] * vx + m[9] * vy + m[10] * vz + m[11];
        double u = cam->fx * (X / Z) + cam->cx;
        double v = cam->fy * (Y / Z) + cam->cy;
        int bad = !(Z >= cam->z_near) || isnan(u) || isnan(v);
        if (uv) { uv[2 * i] = u; uv[2 * i + 1] = v; }
        flags[i] = (uint8_t)bad;
        if (bad) {
            snapped[2 * i] = 0;
            snapped[2 * i + 1] = 0;
        } else {
            snapped[2 * i] = (int32_t)nearbyint(256.0 * clampd(u, -TKO_GUARD, TKO_GUARD));
            snapped[2 * i + 1] = (int32_t)nearbyint(256.0 * clampd(v, -TKO_GUARD, TKO_GUARD));
        }
    }
}

void tko_keypoints(const double M[4][12], const tko_chain* ch, const tko_camera* cam, double kp[4][2]) {
    for (int j = 0; j < 4; j++) {
        const double* m = M[(int)ch->keypoints[j][3]];
        double vx = ch->keypoints[j][0], vy = ch->keypoints[j][1], vz = ch->keypoints[j][2];
        double X = m[0] * vx + m[1] * vy + m[2] * vz + m[3];
        double Y = m[4] * vx + m[5] * vy + m[6] * vz + m[7];
        double Z = m[8] * vx + m[9] * vy + m[10] * vz + m[11];
        if (!(Z >= cam->z_near)) {
            kp[j][0] = kp[j][1] = NAN;
        } else {
            kp[j][0] = cam->fx * (X / Z) + cam->cx;
            kp[j][1] = cam->fy * (Y / Z) + cam->cy;
        }
    }
}

/* ---- raster: exact integer edge functions, top-left fill rule ---- */
static int64_t floor_div(int64_t a, int64_t b) { /* b > 0 */
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) q -= 1;
    return q;
}

int64_t tko_raster(const int32_t* snapped, const uint8_t* flags, int32_t V,
                   const int32_t* tris, int32_t T, int32_t W, int32_t H,
                   uint64_t* mask, int32_t* counts) {
    (void)V;
    int64_t kept = 0;
    int64_t words_x = (W + 7) / 8;
    for (int32_t t = 0; t < T; t++) {
        int32_t i0 = tris[3 * t], i1 = tris[3 * t + 1], i2 = tris[3 * t + 2];
        if (flags[i0] || flags[i1] || flags[i2]) continue;
        int64_t px[3] = {snapped[2 * i0], snapped[2 * i1], snapped[2 * i2]};
        int64_t py[3] = {snapped[2 * i0 + 1], snapped[2 * i1 + 1], snapped[2 * i2 + 1]};
        int64_t area2 = (px[1] - px[0]) * (py[2] - py[0]) - (py[1] - py[0]) * (px[2] - px[0]);
        if (area2 == 0) continue;
        if (area2 < 0) { /* swap b and c so that the triangle is positively oriented */
            int64_t tx = px[1], ty = py[1];
            px[1] = px[2]; py[1] = py[2];
            px[2] = tx; py[2] = ty;
        }
        int64_t dx[3], dy[3], bias[3];
        for (int e = 0; e < 3; e++) {
            int n = (e + 1) % 3;
            dx[e] = px[n] - px[e];
            dy[e] = py[n] - py[e];
            int top_left = (dy[e] < 0) || (dy[e] == 0 && dx[e] > 0);
            bias[e] = top_left ? 0 : -1;
        }
        int64_t xmin = px[0], xmax = px[0], ymin = py[0], ymax = py[0];
        for (int k = 1; k < 3; k++) {
            if (px[k] < xmin) xmin = px[k];
            if (px[k] > xmax) xmax = px[k];
            if (py[k] < ymin) ymin = py[k];
            if (py[k] > ymax) ymax = py[k];
        }
        /* pixel centres 256*p + 128 inside [min, max] */
        int64_t x0 = -floor_div(-(xmin - 128), 256), x1 = floor_div(xmax - 128, 256);
        int64_t y0 = -floor_div(-(ymin - 128), 256), y1 = floor_div(ymax - 128, 256);
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > W - 1) x1 = W - 1;
        if (y1 > H - 1) y1 = H - 1;
        kept++;
        for (int64_t y = y0; y <= y1; y++) {
            int64_t cy = 256 * y + 128;
            for (int64_t x = x0; x <= x1; x++) {
                int64_t cx = 256 * x + 128;
                int inside = 1;
                for (int e = 0; e < 3; e++) {
                    int64_t E = dx[e] * (cy - py[e]) - dy[e] * (cx - px[e]);
                    if (E + bias[e] < 0) { inside = 0; break; }
                }
                if (!inside) continue;
                mask[(y / 8) * words_x + x / 8] |= (uint64_t)1 << ((y % 8) * 8 + (x % 8));
                if (counts) counts[y * W + x] += 1;
            }
        }
    }
    return kept;
}

void tko_counts(const uint64_t* S, const uint64_t* M, int32_t W, int32_t H, int64_t out[3]) {
    int64_t a = 0, i = 0, m = 0;
    int64_t wx = (W + 7) / 8;
    for (int32_t y = 0; y < H; y++)
        for (int32_t x = 0; x < W; x++) {
            int64_t w = (y / 8) * wx + x / 8;
            int b = (y % 8) * 8 + (x % 8);
            int s = (int)((S[w] >> b) & 1u), t = (int)((M[w] >> b) & 1u);
            a += s;
            m += t;
            i += s & t;
        }
    out[0] = a; out[1] = i; out[2] = m;
}

double tko_mask_loss(int64_t a, int64_t i, int64_t m, int32_t kind, double lambda_app) {
    if (kind == 0) {
        int64_t uni = a + m - i;
        if (uni == 0) return 0.0;
        return 1.0 - (double)i / (double)uni;
    }
    return (double)(a + m - 2 * i) + lambda_app * fabs((double)(a - m));
}

static double dist2(const double a[2], const double b[2]) {
    return sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]));
}
/* positive part; NaN propagates so that an invalid candidate ranks last */
static double pos(double x) { return isnan(x) ? x : (x > 0.0 ? x : 0.0); }

double tko_kp_loss(const double kp[4][2], const double ref[4][2], double tau) {
    double fixed = pos(dist2(kp[0], ref[0]) - tau) + pos(dist2(kp[1], ref[1]) - tau);
    double keep = pos(dist2(kp[2], ref[2]) - tau) + pos(dist2(kp[3], ref[3]) - tau);
    double swap = pos(dist2(kp[2], ref[3]) - tau) + pos(dist2(kp[3], ref[2]) - tau);
    double mp[2] = {0.5 * (kp[2][0] + kp[3][0]), 0.5 * (kp[2][1] + kp[3][1])};
    double mr[2] = {0.5 * (ref[2][0] + ref[3][0]), 0.5 * (ref[2][1] + ref[3][1])};
    double tips = keep < swap ? keep : swap;
    if (isnan(keep) || isnan(swap)) tips = NAN;
    return fixed + tips + pos(dist2(mp, mr) - tau);
}

/* Eq. (8) as printed, on the two tool tips (keypoints 2, 3): the better of the
 * two assignments of the detected tips plus the tip-midpoint term, each as
 * (distance - tau)_+; 0 unless exactly two distinct reference tips exist
 * (both finite and not the same point). */
double tko_kp_loss_tips(const double kp[4][2], const double ref[4][2], double tau) {
    if (!(isfinite(ref[2][0]) && isfinite(ref[2][1]) && isfinite(ref[3][0]) && isfinite(ref[3][1])))
        return 0.0;
    if (ref[2][0] == ref[3][0] && ref[2][1] == ref[3][1]) return 0.0;
    double keep = pos(dist2(kp[2], ref[2]) - tau) + pos(dist2(kp[3], ref[3]) - tau);
    double swap = pos(dist2(kp[2], ref[3]) - tau) + pos(dist2(kp[3], ref[2]) - tau);
    double tips = keep < swap ? keep : swap;
    if (isnan(keep) || isnan(swap)) tips = NAN;
    double mp[2] = {0.5 * (kp[2][0] + kp[3][0]), 0.5 * (kp[2][1] + kp[3][1])};
    double mr[2] = {0.5 * (ref[2][0] + ref[3][0]), 0.5 * (ref[2][1] + ref[3][1])};
    return tips + pos(dist2(mp, mr) - tau);
}

/* ---- whole-candidate evaluation (CPU baseline) ---- */
int32_t tko_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void tko_eval_batch(const double* theta, int32_t batch, int32_t n_arms, const tko_chain* chains,
                    const tko_mesh* meshes, const tko_camera* cam, const uint64_t* target,
                    int64_t* counts, uint64_t* masks_out, int32_t n_threads) {
    int32_t W = cam->width, H = cam->height;
    int64_t words = (int64_t)((H + 7) / 8) * ((W + 7) / 8);
    int32_t vmax = 0;
    for (int a = 0; a < n_arms; a++)
        if (meshes[a].n_vertices > vmax) vmax = meshes[a].n_vertices;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
#endif
    for (int32_t b = 0; b < batch; b++) {
        uint64_t* mask = (uint64_t*)calloc((size_t)words, sizeof(uint64_t));
        int32_t* snapped = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(vmax > 0 ? vmax : 1));
        uint8_t* flags = (uint8_t*)malloc((size_t)(vmax > 0 ? vmax : 1));
        for (int a = 0; a < n_arms; a++) {
            double M[4][12];
            tko_fk(theta + ((int64_t)b * n_arms + a) * 9, &chains[a], M);
            tko_project_snap((const double(*)[12])M, meshes[a].vertices, meshes[a].vertex_link,
                             meshes[a].n_vertices, cam, NULL, snapped, flags);
            tko_raster(snapped, flags, meshes[a].n_vertices, meshes[a].triangles, meshes[a].n_triangles,
                       W, H, mask, NULL);
        }
        int64_t c[3];
        tko_counts(mask, target, W, H, c);
        counts[2 * b] = c[0];
        counts[2 * b + 1] = c[1];
        if (masks_out) memcpy(masks_out + (int64_t)b * words, mask, sizeof(uint64_t) * (size_t)words);
        free(mask);
        free(snapped);
        free(flags);
    }
    (void)n_threads;
}
