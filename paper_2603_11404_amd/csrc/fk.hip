// Forward kinematics of the candidates and loss composition.
//
// FK (paper Sec. III-A.3): cosine joint map qhat -> q in [lb, ub]; look-at
// rotation R = Ry(gamma) Rx(alpha) Rz(beta) with translation (x, y, z) gives
// T_r^c; the link chain T_l(q) of the instrument gives M_l = T_r^c T_l, the
// transform applied to the mesh vertices of link l by the renderer
// S = R(K(Pi(T_r^c T_m^r(q) v_m))) of Sec. III-A.2.  One thread per
// (candidate, arm), FP64 internally, FP32 output.
//
// Loss (Eq. objective, Eq. render_loss, Eq. kpts_loss; mask error 1 - IoU of
// Sec. IV): one thread per candidate, FP64 from integer counts.
#include <cmath>
#include <cstring>

#include "tk_internal.h"

namespace tk {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct ChainK {
    double d, lb[3], ub[3], kp[4][4];
};

struct FkArgs {
    ChainK ch[kMaxArms];
    CamK cam;
    int32_t batch, n_arms;
};

// 3x4 affine [R|t] product C = A * B
__device__ inline void aff_mul(const double* A, const double* B, double* C) {
    double t[12];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 4; j++) {
            double s = A[4 * i + 0] * B[0 + j] + A[4 * i + 1] * B[4 + j] + A[4 * i + 2] * B[8 + j];
            if (j == 3) s += A[4 * i + 3];
            t[4 * i + j] = s;
        }
    for (int i = 0; i < 12; i++) C[i] = t[i];
}

__device__ inline double decode_joint(double qh, double lb, double ub) {
    return lb + (ub - lb) / 2.0 * (1.0 - cos(kPi * (qh - lb) / (ub - lb)));
}

__global__ __launch_bounds__(256) void fk_kernel(const float* __restrict__ X, FkArgs a, float* __restrict__ link_xf,
                                                 float* __restrict__ kp) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.batch * a.n_arms) return;
    const int b = idx / a.n_arms, arm = idx % a.n_arms;
    const ChainK ch = arm == 0 ? a.ch[0] : a.ch[1];   // selected, not indexed: keeps the chain in registers
    const float* th = X + (size_t(b) * a.n_arms + arm) * 9;
    const double al = th[0], be = th[1], ga = th[2];

    // R = Ry(gamma) Rx(alpha) Rz(beta)
    double sa, ca, sb, cb, sg, cg;
    sincos(al, &sa, &ca);
    sincos(be, &sb, &cb);
    sincos(ga, &sg, &cg);
    // Ry * Rx
    const double RyRx[9] = {cg, sg * sa, sg * ca, 0.0, ca, -sa, -sg, cg * sa, cg * ca};
    double T[12];
    for (int i = 0; i < 3; i++) {
        T[4 * i + 0] = RyRx[3 * i + 0] * cb + RyRx[3 * i + 1] * sb;
        T[4 * i + 1] = -RyRx[3 * i + 0] * sb + RyRx[3 * i + 1] * cb;
        T[4 * i + 2] = RyRx[3 * i + 2];
    }
    T[3] = th[3];
    T[7] = th[4];
    T[11] = th[5];

    double q[3];
    for (int j = 0; j < 3; j++) q[j] = decode_joint(double(th[6 + j]), ch.lb[j], ch.ub[j]);
    double s1, c1;
    sincos(q[0], &s1, &c1);
    const double pitch[12] = {1, 0, 0, 0, 0, c1, -s1, 0, 0, s1, c1, 0};
    double M[4][12];
    // shaft: T_0 = I
    for (int e = 0; e < 12; e++) M[0][e] = T[e];
    // wrist: Rx(q1)
    aff_mul(T, pitch, M[1]);
    // jaws: Rx(q1) Tr(0,0,d) Ry(q2 +- q3/2)
    const double yaw_origin[12] = {1, 0, 0, 0, 0, c1, -s1, -s1 * ch.d, 0, s1, c1, c1 * ch.d};
    double TY[12];
    aff_mul(T, yaw_origin, TY);
    for (int side = 0; side < 2; side++) {
        const double phi = side == 0 ? q[1] + 0.5 * q[2] : q[1] - 0.5 * q[2];
        double sp, cp;
        sincos(phi, &sp, &cp);
        const double ry[12] = {cp, 0, sp, 0, 0, 1, 0, 0, -sp, 0, cp, 0};
        aff_mul(TY, ry, M[2 + side]);
    }
    float* out = link_xf + (size_t(b) * a.n_arms + arm) * 48;
#pragma unroll
    for (int l = 0; l < 4; l++)
#pragma unroll
        for (int e = 0; e < 12; e++) out[12 * l + e] = float(M[l][e]);

    if (kp) {
        float* o = kp + (size_t(b) * a.n_arms + arm) * 8;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int link = int(ch.kp[j][3]);
            double m[12];
#pragma unroll
            for (int e = 0; e < 12; e++)
                m[e] = link == 0 ? M[0][e] : link == 1 ? M[1][e] : link == 2 ? M[2][e] : M[3][e];
            const double vx = ch.kp[j][0], vy = ch.kp[j][1], vz = ch.kp[j][2];
            const double Xc = m[0] * vx + m[1] * vy + m[2] * vz + m[3];
            const double Yc = m[4] * vx + m[5] * vy + m[6] * vz + m[7];
            const double Zc = m[8] * vx + m[9] * vy + m[10] * vz + m[11];
            if (!(Zc >= double(a.cam.z_near))) {
                o[2 * j] = NAN;
                o[2 * j + 1] = NAN;
            } else {
                o[2 * j] = float(double(a.cam.fx) * (Xc / Zc) + double(a.cam.cx));
                o[2 * j + 1] = float(double(a.cam.fy) * (Yc / Zc) + double(a.cam.cy));
            }
        }
    }
}

// ---------------------------------------------------------------- loss composition

struct LossArgs {
    double lambda_app, lambda_kp, tau;
    int32_t batch, kind, n_arms;
};

__device__ inline double posp(double x) { return x != x ? x : (x > 0.0 ? x : 0.0); }

__device__ inline double dist(const float* p, const float* r) {
    const double dx = double(p[0]) - double(r[0]), dy = double(p[1]) - double(r[1]);
    return sqrt(dx * dx + dy * dy);
}

__global__ __launch_bounds__(256) void compose_loss_kernel(const int32_t* __restrict__ counts,
                                                           const int32_t* __restrict__ target_count,
                                                           const float* __restrict__ kp,
                                                           const float* __restrict__ kp_ref, LossArgs a,
                                                           double* __restrict__ loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.batch) return;
    const int64_t s_cnt = counts[2 * b], inter = counts[2 * b + 1], m = *target_count;
    double L;
    if (a.kind == 0) {
        const int64_t uni = s_cnt + m - inter;
        L = uni == 0 ? 0.0 : 1.0 - double(inter) / double(uni);
    } else {
        L = double(s_cnt + m - 2 * inter) + a.lambda_app * fabs(double(s_cnt - m));
    }
    if (kp && kp_ref && a.lambda_kp != 0.0) {
        for (int arm = 0; arm < a.n_arms; arm++) {
            const float* p = kp + (size_t(b) * a.n_arms + arm) * 8;
            const float* r = kp_ref + size_t(arm) * 8;
            const double fixed = posp(dist(p + 0, r + 0) - a.tau) + posp(dist(p + 2, r + 2) - a.tau);
            const double keep = posp(dist(p + 4, r + 4) - a.tau) + posp(dist(p + 6, r + 6) - a.tau);
            const double swap = posp(dist(p + 4, r + 6) - a.tau) + posp(dist(p + 6, r + 4) - a.tau);
            double tips = keep < swap ? keep : swap;
            if (keep != keep || swap != swap) tips = NAN;
            const double mpx = 0.5 * (double(p[4]) + double(p[6])), mpy = 0.5 * (double(p[5]) + double(p[7]));
            const double mrx = 0.5 * (double(r[4]) + double(r[6])), mry = 0.5 * (double(r[5]) + double(r[7]));
            const double mid = posp(sqrt((mpx - mrx) * (mpx - mrx) + (mpy - mry) * (mpy - mry)) - a.tau);
            L += a.lambda_kp * (fixed + tips + mid);
        }
    }
    loss[b] = L;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_fk_transform(const float* d_X, int32_t batch, int32_t n_arms, const tk_chain* chains, float* d_link_xf,
                          float* d_kp, const tk_camera* cam, tk_stream s) {
    clear_error();
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    TK_REQUIRE(n_arms >= 1 && n_arms <= kMaxArms, "n_arms = %d outside 1..%d", n_arms, kMaxArms);
    TK_REQUIRE(chains != nullptr, "chains is NULL");
    TK_REQUIRE(batch == 0 || (d_X != nullptr && d_link_xf != nullptr), "X / link_xf is NULL");
    FkArgs a;
    std::memset(&a, 0, sizeof a);
    if (d_kp) {
        if (tk_status st = validate_camera(cam)) return st;
        a.cam = make_cam(*cam);
    }
    for (int i = 0; i < n_arms; i++) {
        const tk_chain& c = chains[i];
        TK_REQUIRE(std::isfinite(c.d_pitch_yaw), "chain %d: d_pitch_yaw not finite", i);
        a.ch[i].d = c.d_pitch_yaw;
        for (int j = 0; j < 3; j++) {
            TK_REQUIRE(c.q_ub[j] > c.q_lb[j], "chain %d: joint %d has q_ub <= q_lb", i, j);
            a.ch[i].lb[j] = c.q_lb[j];
            a.ch[i].ub[j] = c.q_ub[j];
        }
        for (int j = 0; j < 4; j++) {
            TK_REQUIRE(c.keypoints[j][3] >= 0 && c.keypoints[j][3] <= 3 &&
                           c.keypoints[j][3] == double(int(c.keypoints[j][3])),
                       "chain %d: keypoint %d has invalid link id", i, j);
            for (int e = 0; e < 4; e++) a.ch[i].kp[j][e] = c.keypoints[j][e];
        }
    }
    a.batch = batch;
    a.n_arms = n_arms;
    if (batch == 0) return TK_OK;
    const int total = batch * n_arms, threads = 256;
    hipLaunchKernelGGL(fk_kernel, dim3((total + threads - 1) / threads), dim3(threads), 0,
                       reinterpret_cast<hipStream_t>(s), d_X, a, d_link_xf, d_kp);
    return check_launch("tk_fk_transform");
}

tk_status tk_compose_loss(const int32_t* d_counts, int32_t batch, const int32_t* d_target_count, int32_t kind,
                          double lambda_app, const float* d_kp, const float* d_kp_ref, int32_t n_arms,
                          double lambda_kp, double tau, double* d_loss, tk_stream s) {
    clear_error();
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    TK_REQUIRE(kind == 0 || kind == 1, "kind = %d must be 0 (1 - IoU) or 1 (render loss)", kind);
    TK_REQUIRE(batch == 0 || (d_counts && d_target_count && d_loss), "counts / target_count / loss is NULL");
    TK_REQUIRE(std::isfinite(lambda_app) && std::isfinite(lambda_kp) && std::isfinite(tau), "non-finite weights");
    TK_REQUIRE((d_kp == nullptr) == (d_kp_ref == nullptr), "kp and kp_ref must both be given or both NULL");
    TK_REQUIRE(d_kp == nullptr || (n_arms >= 1 && n_arms <= kMaxArms), "n_arms = %d outside 1..%d", n_arms,
               kMaxArms);
    if (batch == 0) return TK_OK;
    LossArgs a{lambda_app, lambda_kp, tau, batch, kind, n_arms};
    const int threads = 256;
    hipLaunchKernelGGL(compose_loss_kernel, dim3((batch + threads - 1) / threads), dim3(threads), 0,
                       reinterpret_cast<hipStream_t>(s), d_counts, d_target_count, d_kp, d_kp_ref, a, d_loss);
    return check_launch("tk_compose_loss");
}

}  // extern "C"
