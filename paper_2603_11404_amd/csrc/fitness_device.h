// Device functions shared by the stand-alone FK / loss kernels and the fused
// CMA-ES tell-ask kernel, so that both paths produce identical bits.
#pragma once

#include "tk_internal.h"

namespace tk {

// 3x4 affine [R|t] product C = A * B (row-major)
__device__ __forceinline__ void aff_mul(const float* A, const float* B, float* C) {
    float t[12];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float s = A[4 * i + 0] * B[0 + j] + A[4 * i + 1] * B[4 + j] + A[4 * i + 2] * B[8 + j];
            if (j == 3) s += A[4 * i + 3];
            t[4 * i + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 12; i++) C[i] = t[i];
}

// Cosine joint map (Sec. III-A.3): unconstrained qhat -> q in [lb, ub].
__device__ __forceinline__ float decode_joint(float qh, float lb, float ub) {
    constexpr float kPiF = 3.14159265358979323846f;
    return lb + (ub - lb) * 0.5f * (1.0f - cosf(kPiF * (qh - lb) / (ub - lb)));
}

// Forward kinematics in FP32 (Sec. III-A.3 and the renderer input
// T_r^c T_m^r(q) of Sec. III-A.2), in three pieces so that lanes can share
// the work of one candidate and still compute every output with the same
// operations: the pose T_r^c and joint angles, one link transform
// M_l = T_r^c T_l(q) (shaft, wrist, jaw+, jaw-), one projected keypoint.
struct FkPose {
    float T[12];   // T_r^c, 3x4 row-major
    float q[3];    // decoded joint angles
    float s1, c1;  // sin, cos of q1
};

// The pose from its trigonometric inputs: sines and cosines of the angles
// alpha, beta, gamma (th[0..2]), the decoded joints q and sin, cos of q1.
__device__ __forceinline__ void fk_pose_from(const float* __restrict__ th, float sa, float ca, float sb, float cb,
                                             float sg, float cg, const float* __restrict__ q, float s1, float c1,
                                             FkPose& P) {
    // R = Ry(gamma) Rx(alpha) Rz(beta)
    const float RyRx[9] = {cg, sg * sa, sg * ca, 0.0f, ca, -sa, -sg, cg * sa, cg * ca};
#pragma unroll
    for (int i = 0; i < 3; i++) {
        P.T[4 * i + 0] = RyRx[3 * i + 0] * cb + RyRx[3 * i + 1] * sb;
        P.T[4 * i + 1] = -RyRx[3 * i + 0] * sb + RyRx[3 * i + 1] * cb;
        P.T[4 * i + 2] = RyRx[3 * i + 2];
    }
    P.T[3] = th[3];
    P.T[7] = th[4];
    P.T[11] = th[5];
#pragma unroll
    for (int j = 0; j < 3; j++) P.q[j] = q[j];
    P.s1 = s1;
    P.c1 = c1;
}

__device__ __forceinline__ void fk_pose(const float* __restrict__ th, const ChainK& ch, FkPose& P) {
    float sa, ca, sb, cb, sg, cg;
    sincosf(th[0], &sa, &ca);
    sincosf(th[1], &sb, &cb);
    sincosf(th[2], &sg, &cg);
    float q[3];
#pragma unroll
    for (int j = 0; j < 3; j++) q[j] = decode_joint(th[6 + j], ch.lb[j], ch.ub[j]);
    float s1, c1;
    sincosf(q[0], &s1, &c1);
    fk_pose_from(th, sa, ca, sb, cb, sg, cg, q, s1, c1, P);
}

// Angle phi of link l's last factor Ry(phi): q2 + q3 / 2 and q2 - q3 / 2 for
// the jaws, 0 below them.
__device__ __forceinline__ float fk_link_phi(int l, const float* __restrict__ q) {
    return l == 2 ? q[1] + 0.5f * q[2] : l == 3 ? q[1] - 0.5f * q[2] : 0.0f;
}

// Link l: 0 shaft (T_0 = I), 1 wrist Rx(q1), 2 / 3 jaws Rx(q1) Tr(0, 0, d) Ry(q2 +- q3 / 2).
// One form for every link, M = T_r^c [Rx(q1) | Tr(0, 0, d)] Ry(phi), with
// q1 = 0 for the shaft, d = 0 below the jaws and phi = 0 below them: the
// factors are then exact identities (products with 1 and 0, sums with 0), so
// every link gets the bits of its own formula (up to the sign of zeros), and
// lanes holding different links take one path instead of three.  sp, cp:
// sin and cos of fk_link_phi(l, P.q).
__device__ __forceinline__ void fk_link_from(int l, const FkPose& P, const ChainK& ch, float sp, float cp,
                                             float* __restrict__ M) {
    const float s1 = l >= 1 ? P.s1 : 0.0f, c1 = l >= 1 ? P.c1 : 1.0f;
    const float d = l >= 2 ? ch.d : 0.0f;
    const float yaw_origin[12] = {1, 0, 0, 0, 0, c1, -s1, -s1 * d, 0, s1, c1, c1 * d};
    float TY[12];
    aff_mul(P.T, yaw_origin, TY);
    const float ry[12] = {cp, 0, sp, 0, 0, 1, 0, 0, -sp, 0, cp, 0};
    aff_mul(TY, ry, M);
}

__device__ __forceinline__ void fk_link(int l, const FkPose& P, const ChainK& ch, float* __restrict__ M) {
    float sp, cp;
    sincosf(fk_link_phi(l, P.q), &sp, &cp);
    fk_link_from(l, P, ch, sp, cp, M);
}

// Element j (0..3) of four values, chosen without indexing (a per-lane index
// into a struct would move the struct to private memory).
template <typename T>
__device__ __forceinline__ T select4(int j, T v0, T v1, T v2, T v3) {
    return j == 0 ? v0 : j == 1 ? v1 : j == 2 ? v2 : v3;
}

// Keypoint j of the chain, given the transform M of its link: pinhole
// projection, NaN behind the near plane.
__device__ __forceinline__ void fk_keypoint(const float* __restrict__ M, const ChainK& ch, int j, const CamK& cam,
                                            float* __restrict__ kp2) {
    const float vx = select4(j, ch.kp[0][0], ch.kp[1][0], ch.kp[2][0], ch.kp[3][0]);
    const float vy = select4(j, ch.kp[0][1], ch.kp[1][1], ch.kp[2][1], ch.kp[3][1]);
    const float vz = select4(j, ch.kp[0][2], ch.kp[1][2], ch.kp[2][2], ch.kp[3][2]);
    const float Xc = M[0] * vx + M[1] * vy + M[2] * vz + M[3];
    const float Yc = M[4] * vx + M[5] * vy + M[6] * vz + M[7];
    const float Zc = M[8] * vx + M[9] * vy + M[10] * vz + M[11];
    if (!(Zc >= cam.z_near)) {
        kp2[0] = NAN;
        kp2[1] = NAN;
    } else {
        kp2[0] = cam.fx * (Xc / Zc) + cam.cx;
        kp2[1] = cam.fy * (Yc / Zc) + cam.cy;
    }
}

// Whole forward kinematics of one candidate and arm: th = (alpha, beta,
// gamma, x, y, z, qhat1..3) -> out[4][12], and the four keypoints into kp
// (when not NULL).
__device__ __forceinline__ void fk_candidate(const float* __restrict__ th, const ChainK& ch, const CamK& cam,
                                             float* __restrict__ out, float* __restrict__ kp) {
    FkPose P;
    fk_pose(th, ch, P);
    float M[4][12];
#pragma unroll
    for (int l = 0; l < 4; l++) fk_link(l, P, ch, M[l]);
#pragma unroll
    for (int l = 0; l < 4; l++)
#pragma unroll
        for (int e = 0; e < 12; e++) out[12 * l + e] = M[l][e];
    if (kp) {
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int link = ch.kp_link[j];
            float m[12];
#pragma unroll
            for (int e = 0; e < 12; e++)
                m[e] = link == 0 ? M[0][e] : link == 1 ? M[1][e] : link == 2 ? M[2][e] : M[3][e];
            fk_keypoint(m, ch, j, cam, kp + 2 * j);
        }
    }
}

// ---------------------------------------------------------------- loss

__device__ __forceinline__ double pos_part(double x) { return x != x ? x : (x > 0.0 ? x : 0.0); }

__device__ __forceinline__ double kp_dist(const float* p, const float* r) {
    const double dx = double(p[0]) - double(r[0]), dy = double(p[1]) - double(r[1]);
    return sqrt(dx * dx + dy * dy);
}

// Loss of one candidate in FP64 from its counts (Eq. (5), (6), (8); mask error
// 1 - IoU of Sec. IV):
//   kind 0: 1 - i / (a + m - i), 0 when the union is empty;
//   kind 1: (a + m - 2i) + lambda_app |a - m|;
// plus lambda_kp times the keypoint term of every arm when kp is given: the
// shaft and wrist keypoints' (|p - r| - tau)_+, the better assignment of the
// two jaw tips, and the tip midpoint; with the TK_KP_TWO_TIPS bit in kind,
// Eq. (8) as printed instead: the two jaw tips and their midpoint only, and no
// term for an arm whose two reference tips are not finite and distinct.
// kp: this candidate's [n_arms][4][2].
__device__ __forceinline__ double compose_loss_one(int64_t a_cnt, int64_t inter, int64_t m, const float* kp,
                                                   const float* kp_ref, const LossArgs& la) {
    double L;
    if ((la.kind & 15) == 0) {
        const int64_t uni = a_cnt + m - inter;
        L = uni == 0 ? 0.0 : 1.0 - double(inter) / double(uni);
    } else {
        L = double(a_cnt + m - 2 * inter) + la.lambda_app * fabs(double(a_cnt - m));
    }
    if (kp && kp_ref && la.lambda_kp != 0.0) {
        for (int arm = 0; arm < la.n_arms; arm++) {
            const float* p = kp + arm * 8;
            const float* r = kp_ref + arm * 8;
            const bool two_tips = (la.kind & TK_KP_TWO_TIPS) != 0;
            if (two_tips && !(isfinite(r[4]) && isfinite(r[5]) && isfinite(r[6]) && isfinite(r[7]) &&
                              !(r[4] == r[6] && r[5] == r[7])))
                continue;
            const double fixed = two_tips ? 0.0
                                          : pos_part(kp_dist(p + 0, r + 0) - la.tau) +
                                                pos_part(kp_dist(p + 2, r + 2) - la.tau);
            const double keep = pos_part(kp_dist(p + 4, r + 4) - la.tau) + pos_part(kp_dist(p + 6, r + 6) - la.tau);
            const double swap = pos_part(kp_dist(p + 4, r + 6) - la.tau) + pos_part(kp_dist(p + 6, r + 4) - la.tau);
            double tips = keep < swap ? keep : swap;
            if (keep != keep || swap != swap) tips = NAN;
            const double mpx = 0.5 * (double(p[4]) + double(p[6])), mpy = 0.5 * (double(p[5]) + double(p[7]));
            const double mrx = 0.5 * (double(r[4]) + double(r[6])), mry = 0.5 * (double(r[5]) + double(r[7]));
            const double mid = pos_part(sqrt((mpx - mrx) * (mpx - mrx) + (mpy - mry) * (mpy - mry)) - la.tau);
            L += la.lambda_kp * (fixed + tips + mid);
        }
    }
    return L;
}

}  // namespace tk
