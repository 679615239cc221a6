/*
 * tko_soft.c -- oracle of the soft (differentiable) silhouette and of the
 * forward-kinematics Jacobian.  TEST INFRASTRUCTURE ONLY (see tko.h).
 *
 * The soft silhouette is the differentiable stand-in for the renderer
 * S = R(K(Pi(T_r^c T_m^r(q) v_m))) of Sec. III-A.2, and its loss is the
 * squared-error term of Eq. (6) summed over the pixels.  Definitions, written
 * out literally in FP64 (no snapping, no fixed point):
 *   - pixel (x, y) has its centre at (x + 0.5, y + 0.5);
 *   - a face takes part when all three vertices lie in front of z_near and its
 *     projected area is not zero;
 *   - d_j(p): signed Euclidean distance from the pixel centre to the boundary
 *     of face j, positive inside, the smallest of the three point-to-segment
 *     distances;
 *   - prob_j(p) = (sig(d_j / sigma) - s0) / (1 - s0) for d_j >= -10 sigma and 0
 *     below, with sig the logistic function and s0 = sig(-10): the logistic
 *     of the distance, shifted so that it reaches 0 exactly at the cutoff;
 *   - S(p) = 1 - prod_j (1 - prob_j(p)) over the faces of every arm
 *     (probabilistic OR);
 *   - L = sum over the pixels of (S(p) - M(p))^2, M the observed mask.
 * The gradient is the chain rule written term by term: the product over the
 * other faces, the derivative of prob_j in d_j, of d_j in the two end points
 * of the nearest edge, of the pinhole projection in the camera-frame vertex,
 * and of the link transform in theta (tko_fk_jacobian, including the cosine
 * joint map).
 */
#include "tko.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TKS_PI 3.14159265358979323846

/* ---- elementary rotations and their derivatives ---- */
static void rx(double a, double R[9], double dR[9]) {
    double c = cos(a), s = sin(a);
    double r[9] = {1, 0, 0, 0, c, -s, 0, s, c};
    double d[9] = {0, 0, 0, 0, -s, -c, 0, c, -s};
    memcpy(R, r, sizeof r);
    memcpy(dR, d, sizeof d);
}
static void ry(double a, double R[9], double dR[9]) {
    double c = cos(a), s = sin(a);
    double r[9] = {c, 0, s, 0, 1, 0, -s, 0, c};
    double d[9] = {-s, 0, c, 0, 0, 0, -c, 0, -s};
    memcpy(R, r, sizeof r);
    memcpy(dR, d, sizeof d);
}
static void rz(double a, double R[9], double dR[9]) {
    double c = cos(a), s = sin(a);
    double r[9] = {c, -s, 0, s, c, 0, 0, 0, 1};
    double d[9] = {-s, -c, 0, c, -s, 0, 0, 0, 0};
    memcpy(R, r, sizeof r);
    memcpy(dR, d, sizeof d);
}
static void m3(const double A[9], const double B[9], double C[9]) {
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[3 * i + k] * B[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(C, t, sizeof t);
}
/* affine 3x4 [R|t] from rotation and translation */
static void aff(const double R[9], const double t[3], double T[12]) {
    for (int i = 0; i < 3; i++) {
        T[4 * i + 0] = R[3 * i + 0];
        T[4 * i + 1] = R[3 * i + 1];
        T[4 * i + 2] = R[3 * i + 2];
        T[4 * i + 3] = t[i];
    }
}
/* C = A * B for affine maps (applied to homogeneous points) */
static void amul(const double A[12], const double B[12], double C[12]) {
    double t[12];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 4; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[4 * i + k] * B[4 * k + j];
            if (j == 3) s += A[4 * i + 3];
            t[4 * i + j] = s;
        }
    memcpy(C, t, sizeof t);
}
/* derivative of A * B when only B varies: dC = A_rot dB (the translation of A drops out) */
static void amul_lin(const double A[12], const double dB[12], double dC[12]) {
    double t[12];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 4; j++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[4 * i + k] * dB[4 * k + j];
            t[4 * i + j] = s;
        }
    memcpy(dC, t, sizeof t);
}

/* ---- Jacobian of the link transforms M_l(theta) = T_r^c(pose) T_l(q(qhat)) ---- */
void tko_fk_jacobian(const double theta[9], const tko_chain* ch, double dM[9][4][12]) {
    double Rx_[9], dRx[9], Ry_[9], dRy[9], Rz_[9], dRz[9], R[9], tmp[9];
    rx(theta[0], Rx_, dRx);
    rz(theta[1], Rz_, dRz);
    ry(theta[2], Ry_, dRy);
    const double zero3[3] = {0, 0, 0};
    const double tr[3] = {theta[3], theta[4], theta[5]};
    /* pose and its derivatives: R = Ry(gamma) Rx(alpha) Rz(beta) */
    double P[12], dP[6][12];
    m3(Ry_, Rx_, tmp);
    m3(tmp, Rz_, R);
    aff(R, tr, P);
    double dRa[9], dRb[9], dRg[9];
    m3(Ry_, dRx, tmp);
    m3(tmp, Rz_, dRa);           /* d/d alpha */
    m3(Ry_, Rx_, tmp);
    m3(tmp, dRz, dRb);           /* d/d beta */
    m3(dRy, Rx_, tmp);
    m3(tmp, Rz_, dRg);           /* d/d gamma */
    aff(dRa, zero3, dP[0]);
    aff(dRb, zero3, dP[1]);
    aff(dRg, zero3, dP[2]);
    for (int k = 0; k < 3; k++) {
        double e[3] = {0, 0, 0};
        double Z9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        e[k] = 1.0;
        aff(Z9, e, dP[3 + k]);   /* d/d x, y, z */
    }
    /* joint angles from the cosine map and their derivatives in qhat */
    double q[3], dq[3];
    for (int j = 0; j < 3; j++) {
        const double lb = ch->q_lb[j], ub = ch->q_ub[j];
        const double a = TKS_PI * (theta[6 + j] - lb) / (ub - lb);
        q[j] = lb + (ub - lb) / 2.0 * (1.0 - cos(a));
        dq[j] = (TKS_PI / 2.0) * sin(a);
    }
    /* link transforms and their derivatives in q1, q2, q3 */
    double L[4][12], dL[4][3][12];
    memset(dL, 0, sizeof dL);
    {
        const double I9[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        aff(I9, zero3, L[0]);
        double Rq1[9], dRq1[9];
        rx(q[0], Rq1, dRq1);
        aff(Rq1, zero3, L[1]);
        aff(dRq1, zero3, dL[1][0]);
        const double dz[3] = {0, 0, ch->d_pitch_yaw};
        double o[3], d_o[3];     /* yaw origin Rx(q1) (0, 0, d) and its q1 derivative */
        for (int i = 0; i < 3; i++) {
            o[i] = Rq1[3 * i + 2] * dz[2];
            d_o[i] = dRq1[3 * i + 2] * dz[2];
        }
        for (int side = 0; side < 2; side++) {
            const double sgn = side == 0 ? 0.5 : -0.5;
            const double phi = q[1] + sgn * q[2];
            double Rp[9], dRp[9], Rl[9], dRl1[9], dRlp[9];
            ry(phi, Rp, dRp);
            m3(Rq1, Rp, Rl);
            m3(dRq1, Rp, dRl1);
            m3(Rq1, dRp, dRlp);
            aff(Rl, o, L[2 + side]);
            aff(dRl1, d_o, dL[2 + side][0]);
            aff(dRlp, zero3, dL[2 + side][1]);
            for (int e = 0; e < 12; e++) dL[2 + side][2][e] = sgn * dL[2 + side][1][e];
        }
    }
    for (int l = 0; l < 4; l++) {
        for (int k = 0; k < 6; k++) amul(dP[k], L[l], dM[k][l]);
        for (int j = 0; j < 3; j++) {
            amul_lin(P, dL[l][j], dM[6 + j][l]);
            for (int e = 0; e < 12; e++) dM[6 + j][l][e] *= dq[j];
        }
    }
}

/* ---- soft silhouette ---- */

static double sig(double x) { return 1.0 / (1.0 + exp(-x)); }

typedef struct {
    double u[3], v[3];           /* projected corners */
    double du[3][TKO_SOFT_MAXP]; /* d u_c / d theta (all parameters of all arms) */
    double dv[3][TKO_SOFT_MAXP];
} face_t;

/* Signed distance of (px, py) to the triangle boundary; the nearest edge's
 * corners (ia, ib), its parameter t and unit direction (nx, ny) from the
 * closest boundary point to the pixel, and the sign (+1 inside). */
static double signed_dist(const face_t* f, double px, double py, int* ia, int* ib, double* tt, double* nx,
                          double* ny, double* sg) {
    double best = INFINITY;
    for (int e = 0; e < 3; e++) {
        const int a = e, b = (e + 1) % 3;
        const double ex = f->u[b] - f->u[a], ey = f->v[b] - f->v[a];
        const double wx = px - f->u[a], wy = py - f->v[a];
        const double len2 = ex * ex + ey * ey;
        double t = len2 > 0.0 ? (wx * ex + wy * ey) / len2 : 0.0;
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        const double rx_ = wx - t * ex, ry_ = wy - t * ey;
        const double d = sqrt(rx_ * rx_ + ry_ * ry_);
        if (d < best) {
            best = d;
            *ia = a;
            *ib = b;
            *tt = t;
            *nx = d > 0.0 ? rx_ / d : 0.0;
            *ny = d > 0.0 ? ry_ / d : 0.0;
        }
    }
    /* inside: the pixel is on the same side of all three edges */
    double c[3];
    for (int e = 0; e < 3; e++) {
        const int a = e, b = (e + 1) % 3;
        c[e] = (f->u[b] - f->u[a]) * (py - f->v[a]) - (f->v[b] - f->v[a]) * (px - f->u[a]);
    }
    const int inside = (c[0] >= 0 && c[1] >= 0 && c[2] >= 0) || (c[0] <= 0 && c[1] <= 0 && c[2] <= 0);
    *sg = inside ? 1.0 : -1.0;
    return inside ? best : -best;
}

static int mask_bit(const uint64_t* M, int32_t W, int32_t x, int32_t y) {
    const int32_t bx = (W + 7) / 8;
    return (int)((M[(y / 8) * bx + x / 8] >> ((y % 8) * 8 + x % 8)) & 1u);
}

/* The faces that take part, with their projected corners and corner
 * Jacobians (in list order over the arms); *used receives their count. */
static face_t* build_faces(const double* theta, int32_t n_arms, const tko_chain* chains, const tko_mesh* meshes,
                           const tko_camera* cam, int32_t* used_out) {
    int32_t nf = 0;
    for (int a = 0; a < n_arms; a++) nf += meshes[a].n_triangles;
    face_t* F = (face_t*)malloc(sizeof(face_t) * (size_t)(nf > 0 ? nf : 1));
    int32_t used = 0;
    for (int a = 0; a < n_arms; a++) {
        double M[4][12], dM[9][4][12];
        tko_fk(theta + 9 * a, &chains[a], M);
        tko_fk_jacobian(theta + 9 * a, &chains[a], dM);
        const tko_mesh* m = &meshes[a];
        for (int32_t t = 0; t < m->n_triangles; t++) {
            face_t f;
            memset(&f, 0, sizeof f);
            int ok = 1;
            for (int c = 0; c < 3; c++) {
                const int32_t vi = m->triangles[3 * t + c];
                const int l = m->vertex_link[vi];
                const double vx = m->vertices[3 * vi], vy = m->vertices[3 * vi + 1], vz = m->vertices[3 * vi + 2];
                const double* T = M[l];
                const double X = T[0] * vx + T[1] * vy + T[2] * vz + T[3];
                const double Y = T[4] * vx + T[5] * vy + T[6] * vz + T[7];
                const double Z = T[8] * vx + T[9] * vy + T[10] * vz + T[11];
                if (!(Z >= cam->z_near)) ok = 0;
                f.u[c] = cam->fx * (X / Z) + cam->cx;
                f.v[c] = cam->fy * (Y / Z) + cam->cy;
                for (int k = 0; k < 9; k++) {
                    const double* D = dM[k][l];
                    const double dX = D[0] * vx + D[1] * vy + D[2] * vz + D[3];
                    const double dY = D[4] * vx + D[5] * vy + D[6] * vz + D[7];
                    const double dZ = D[8] * vx + D[9] * vy + D[10] * vz + D[11];
                    /* u = fx X / Z + cx: du = fx (dX Z - X dZ) / Z^2 */
                    f.du[c][9 * a + k] = cam->fx * (dX * Z - X * dZ) / (Z * Z);
                    f.dv[c][9 * a + k] = cam->fy * (dY * Z - Y * dZ) / (Z * Z);
                }
            }
            const double area = (f.u[1] - f.u[0]) * (f.v[2] - f.v[0]) - (f.v[1] - f.v[0]) * (f.u[2] - f.u[0]);
            if (ok && area != 0.0 && isfinite(area)) F[used++] = f;
        }
    }
    *used_out = used;
    return F;
}

/* Whether pixel centre (px, py) lies in face f's box grown by 10 sigma (cut =
 * -10 sigma): outside it the distance to the face exceeds 10 sigma. */
static int in_band_box(const face_t* f, double cut, double px, double py) {
    double lo_u = f->u[0], hi_u = f->u[0], lo_v = f->v[0], hi_v = f->v[0];
    for (int c = 1; c < 3; c++) {
        lo_u = fmin(lo_u, f->u[c]); hi_u = fmax(hi_u, f->u[c]);
        lo_v = fmin(lo_v, f->v[c]); hi_v = fmax(hi_v, f->v[c]);
    }
    return !(px < lo_u + cut || px > hi_u - cut || py < lo_v + cut || py > hi_v - cut);
}

double tko_soft(const double* theta, int32_t n_arms, const tko_chain* chains, const tko_mesh* meshes,
                const tko_camera* cam, double sigma, const uint64_t* target, double* S_out, double* grad) {
    const int np = 9 * n_arms;
    /* faces that take part, with their projected corners and corner Jacobians */
    int32_t used = 0;
    face_t* F = build_faces(theta, n_arms, chains, meshes, cam, &used);
    const double s0 = sig(-10.0);
    const double cut = -10.0 * sigma;
    double loss = 0.0;
    if (grad)
        for (int k = 0; k < np; k++) grad[k] = 0.0;
    /* per pixel: the faces within the band, their probabilities and derivatives */
    int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(used > 0 ? used : 1));
    double* pr = (double*)malloc(sizeof(double) * (size_t)(used > 0 ? used : 1));
    double* dpd = (double*)malloc(sizeof(double) * (size_t)(used > 0 ? used : 1));
    double (*dd)[TKO_SOFT_MAXP] = malloc(sizeof(double) * TKO_SOFT_MAXP * (size_t)(used > 0 ? used : 1));
    for (int32_t y = 0; y < cam->height; y++) {
        for (int32_t x = 0; x < cam->width; x++) {
            const double px = x + 0.5, py = y + 0.5;
            int32_t k = 0;
            for (int32_t j = 0; j < used; j++) {
                const face_t* f = &F[j];
                /* outside the face's box grown by 10 sigma the distance exceeds 10 sigma */
                if (!in_band_box(f, cut, px, py)) continue;
                int ia, ib;
                double t, nx, ny, sg;
                const double d = signed_dist(f, px, py, &ia, &ib, &t, &nx, &ny, &sg);
                if (d < cut) continue;
                const double s = sig(d / sigma);
                idx[k] = j;
                pr[k] = (s - s0) / (1.0 - s0);
                dpd[k] = s * (1.0 - s) / (sigma * (1.0 - s0));   /* d prob / d d */
                if (grad) {
                    /* d d / d theta through the nearest edge's end points:
                     * dist = |p - q|, q = e_a + t (e_b - e_a): d dist / d e_a = -n (1 - t), d dist / d e_b = -n t */
                    for (int p = 0; p < np; p++) {
                        const double g = -(nx * ((1.0 - t) * f->du[ia][p] + t * f->du[ib][p]) +
                                           ny * ((1.0 - t) * f->dv[ia][p] + t * f->dv[ib][p]));
                        dd[k][p] = sg * g;
                    }
                }
                k++;
            }
            double prod = 1.0;
            for (int32_t i = 0; i < k; i++) prod *= 1.0 - pr[i];
            const double S = 1.0 - prod;
            const double m = target ? (double)mask_bit(target, cam->width, x, y) : 0.0;
            loss += (S - m) * (S - m);
            if (S_out) S_out[(size_t)y * cam->width + x] = S;
            if (grad) {
                for (int32_t i = 0; i < k; i++) {
                    double others = 1.0;                      /* prod over the other faces */
                    for (int32_t j = 0; j < k; j++)
                        if (j != i) others *= 1.0 - pr[j];
                    const double w = 2.0 * (S - m) * others * dpd[i];
                    for (int p = 0; p < np; p++) grad[p] += w * dd[i][p];
                }
            }
        }
    }
    free(dd);
    free(dpd);
    free(pr);
    free(idx);
    free(F);
    return loss;
}

/* ---- the same silhouette, loss and gradient, face-major ----
 *
 * The definitions of tko_soft evaluated face by face over only the pixel
 * centres of each face's box grown by 10 sigma (the same box test, applied
 * inside a range one pixel wider than the box), so that meshes of tens of
 * thousands of faces at 640 x 480 finish in seconds.  Faces are visited in
 * ascending order, so each pixel multiplies its factors 1 - prob_j in the
 * same order as tko_soft: S and the loss are the same numbers.  A factor that
 * is exactly zero (prob = 1, deep inside a face) is counted instead of
 * multiplied; the product over the other faces of the gradient is then the
 * product of the non-zero factors divided by the face's own factor, or zero
 * when another factor is zero (an identity of the product, with no division
 * by zero). */
double tko_soft_banded(const double* theta, int32_t n_arms, const tko_chain* chains, const tko_mesh* meshes,
                       const tko_camera* cam, double sigma, const uint64_t* target, double* S_out, double* grad) {
    const int np = 9 * n_arms;
    const int32_t W = cam->width, H = cam->height;
    int32_t used = 0;
    face_t* F = build_faces(theta, n_arms, chains, meshes, cam, &used);
    const double s0 = sig(-10.0);
    const double cut = -10.0 * sigma;
    double* prod = (double*)malloc(sizeof(double) * (size_t)W * H);       /* product of the non-zero factors */
    int32_t* zeros = (int32_t*)calloc((size_t)W * H, sizeof(int32_t));   /* factors exactly zero */
    double* wpix = (double*)malloc(sizeof(double) * (size_t)W * H);       /* 2 (S - M) */
    for (size_t i = 0; i < (size_t)W * H; i++) prod[i] = 1.0;
    if (grad)
        for (int p = 0; p < np; p++) grad[p] = 0.0;
    double loss = 0.0;
    /* pass 0: the per-pixel products; pass 1 (gradient only): the chain rule */
    for (int pass = 0; pass < (grad ? 2 : 1); pass++) {
        for (int32_t j = 0; j < used; j++) {
            const face_t* f = &F[j];
            double lo_u = f->u[0], hi_u = f->u[0], lo_v = f->v[0], hi_v = f->v[0];
            for (int c = 1; c < 3; c++) {
                lo_u = fmin(lo_u, f->u[c]); hi_u = fmax(hi_u, f->u[c]);
                lo_v = fmin(lo_v, f->v[c]); hi_v = fmax(hi_v, f->v[c]);
            }
            /* a pixel range one pixel wider than the grown box; the box test decides */
            const double x0 = floor(lo_u + cut - 0.5) - 1.0, x1 = ceil(hi_u - cut - 0.5) + 1.0;
            const double y0 = floor(lo_v + cut - 0.5) - 1.0, y1 = ceil(hi_v - cut - 0.5) + 1.0;
            if (!(x1 >= 0.0 && y1 >= 0.0 && x0 <= W - 1 && y0 <= H - 1)) continue;
            const int32_t xa = x0 < 0.0 ? 0 : (int32_t)x0, xb = x1 > W - 1 ? W - 1 : (int32_t)x1;
            const int32_t ya = y0 < 0.0 ? 0 : (int32_t)y0, yb = y1 > H - 1 ? H - 1 : (int32_t)y1;
            for (int32_t y = ya; y <= yb; y++)
                for (int32_t x = xa; x <= xb; x++) {
                    const double px = x + 0.5, py = y + 0.5;
                    if (!in_band_box(f, cut, px, py)) continue;
                    int ia, ib;
                    double t, nx, ny, sg;
                    const double d = signed_dist(f, px, py, &ia, &ib, &t, &nx, &ny, &sg);
                    if (d < cut) continue;
                    const double sgm = sig(d / sigma);
                    const double fac = 1.0 - (sgm - s0) / (1.0 - s0);
                    const size_t q = (size_t)y * W + x;
                    if (pass == 0) {
                        if (fac == 0.0) zeros[q]++;
                        else prod[q] *= fac;
                        continue;
                    }
                    const int others_zero = zeros[q] - (fac == 0.0 ? 1 : 0) > 0;
                    const double others = others_zero ? 0.0 : (fac == 0.0 ? prod[q] : prod[q] / fac);
                    const double w = wpix[q] * others * (sgm * (1.0 - sgm) / (sigma * (1.0 - s0)));
                    for (int p = 0; p < np; p++) {
                        const double g = -(nx * ((1.0 - t) * f->du[ia][p] + t * f->du[ib][p]) +
                                           ny * ((1.0 - t) * f->dv[ia][p] + t * f->dv[ib][p]));
                        grad[p] += w * sg * g;
                    }
                }
        }
        if (pass == 0)
            for (int32_t y = 0; y < H; y++)
                for (int32_t x = 0; x < W; x++) {
                    const size_t q = (size_t)y * W + x;
                    const double S = 1.0 - (zeros[q] > 0 ? 0.0 : prod[q]);
                    const double m = target ? (double)mask_bit(target, W, x, y) : 0.0;
                    loss += (S - m) * (S - m);
                    wpix[q] = 2.0 * (S - m);
                    if (S_out) S_out[q] = S;
                }
    }
    free(wpix);
    free(zeros);
    free(prod);
    free(F);
    return loss;
}
