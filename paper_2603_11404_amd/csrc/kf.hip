// Temporal filter of the per-frame estimates (Sec. III-A.4): a constant-
// velocity Kalman filter over s_t = [theta_t; theta_dot_t] with the motion
// model of Eq. (kf_motion) and the observation z_t = [I 0] s_t + v_t, whose
// measurement is the CMA-ES estimate of the frame; afterwards the filtered
// coordinates with limits (the joint angles) are clamped.
//
// With the process noise Q made of diagonal n x n blocks and a diagonal R,
// F = [[I, dt I], [0, I]] and H = [I 0] couple coordinate i only with its own
// velocity, so P keeps that block structure from a block-diagonal P0 and the
// 2n-dimensional filter is n independent 2-state filters.  One lane per
// coordinate, FP64.
//
// tk_cmaes_estimate turns the CMA-ES mean into that measurement: the physical
// coordinates offset + scale * m, with the joint coordinates passed through
// the cosine map of Sec. III-A.3 (FP64), so that the filter and its clamp act
// on joint angles.
#include <cmath>
#include <cstring>

#include "tk_internal.h"

namespace tk {
namespace {

constexpr int kKfMax = TK_KF_MAX_N;
constexpr int32_t kKfMagic = 0x464b4b54;  // "TKKF"

// Device-resident filter state (one allocation of tk_kf_state_bytes()).
struct KfState {
    int32_t n, magic;
    int64_t frames;                                        // updates applied so far
    double dt;
    double x[kKfMax], v[kKfMax];                           // filtered state
    double pxx[kKfMax], pxv[kKfMax], pvv[kKfMax];          // 2x2 covariance blocks
    double qpp[kKfMax], qpv[kKfMax], qvv[kKfMax];          // process-noise blocks
    double r[kKfMax];                                      // measurement variances
    double lo[kKfMax], hi[kKfMax];                         // clamp limits
};
static_assert(sizeof(KfState) % 8 == 0, "KfState is copied as 8-byte words");

__global__ __launch_bounds__(64) void kf_init_kernel(KfState init, KfState* __restrict__ st) {
    const double* src = reinterpret_cast<const double*>(&init);
    double* dst = reinterpret_cast<double*>(st);
    for (int w = threadIdx.x; w < int(sizeof(KfState) / 8); w += blockDim.x) dst[w] = src[w];
}

__global__ __launch_bounds__(64) void kf_step_kernel(KfState* __restrict__ st, int32_t n,
                                                     const double* __restrict__ z, double* __restrict__ theta,
                                                     double* __restrict__ theta_next) {
    const int i = threadIdx.x;
    if (i == 0) st->frames += 1;
    if (i >= n) return;
    const double dt = st->dt;
    const double a = st->pxx[i], b = st->pxv[i], c = st->pvv[i];
    // predict: s' = F s, P' = F P F^T + Q
    double x = st->x[i] + dt * st->v[i];
    double v = st->v[i];
    double pxx = a + dt * b + dt * (b + dt * c) + st->qpp[i];
    double pxv = b + dt * c + st->qpv[i];
    double pvv = c + st->qvv[i];
    // update with the measurement (a non-finite one is treated as missing)
    const double zi = z[i];
    if (isfinite(zi)) {
        const double S = pxx + st->r[i];
        const double kx = pxx / S, kv = pxv / S;
        const double y = zi - x;
        x = x + kx * y;
        v = v + kv * y;
        // P = (I - K H) P', symmetrised
        const double nxx = (1.0 - kx) * pxx;
        const double nxv = 0.5 * ((1.0 - kx) * pxv + (pxv - kv * pxx));
        const double nvv = pvv - kv * pxv;
        pxx = nxx;
        pxv = nxv;
        pvv = nvv;
    }
    x = fmin(fmax(x, st->lo[i]), st->hi[i]);
    st->x[i] = x;
    st->v[i] = v;
    st->pxx[i] = pxx;
    st->pxv[i] = pxv;
    st->pvv[i] = pvv;
    if (theta) theta[i] = x;
    if (theta_next) theta_next[i] = fmin(fmax(x + dt * v, st->lo[i]), st->hi[i]);
}

struct EstimateArgs {
    double lb[kKfMax], ub[kKfMax];   // cosine-map limits of the joint coordinates
    int32_t n, lambda;
};

__global__ __launch_bounds__(64) void cmaes_estimate_kernel(const void* __restrict__ blob, EstimateArgs a,
                                                            double* __restrict__ z) {
    const int i = threadIdx.x;
    if (i >= a.n) return;
    StateView S = state_view(const_cast<void*>(blob), a.n, a.lambda);
    double th = S.offset[i] + S.scale[i] * S.mean[i];
    if (i % 9 >= 6) {
        const double lb = a.lb[i], ub = a.ub[i];
        th = lb + (ub - lb) * 0.5 * (1.0 - cos(3.14159265358979323846 * (th - lb) / (ub - lb)));
    }
    z[i] = th;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

size_t tk_kf_state_bytes(int32_t n) {
    return n >= 1 && n <= kKfMax ? (sizeof(KfState) + 255) & ~size_t(255) : 0;
}

tk_status tk_kf_init(void* d_kf, int32_t n, const double* x0, const tk_kf_params* p, tk_stream s) {
    clear_error();
    TK_REQUIRE(n >= 1 && n <= kKfMax, "n = %d outside 1..%d", n, kKfMax);
    TK_REQUIRE(d_kf && x0 && p, "kf / x0 / params is NULL");
    TK_REQUIRE(std::isfinite(p->dt) && p->dt > 0.0, "dt must be finite and > 0");
    KfState k;
    std::memset(&k, 0, sizeof k);
    k.n = n;
    k.magic = kKfMagic;
    k.dt = p->dt;
    for (int i = 0; i < kKfMax; i++) {   // unused coordinates: a valid idle filter
        k.pxx[i] = k.pvv[i] = k.r[i] = 1.0;
        k.lo[i] = -INFINITY;
        k.hi[i] = INFINITY;
    }
    for (int i = 0; i < n; i++) {
        TK_REQUIRE(std::isfinite(x0[i]), "x0[%d] not finite", i);
        TK_REQUIRE(std::isfinite(p->p0_pos[i]) && std::isfinite(p->p0_vel[i]) && p->p0_pos[i] >= 0.0 &&
                       p->p0_vel[i] >= 0.0, "p0_pos / p0_vel[%d] must be finite and >= 0", i);
        const double qpp = p->q_pos[i], qpv = p->q_cross[i], qvv = p->q_vel[i];
        TK_REQUIRE(std::isfinite(qpp) && std::isfinite(qpv) && std::isfinite(qvv) && qpp >= 0.0 && qvv >= 0.0 &&
                       qpv * qpv <= qpp * qvv, "process noise block %d is not finite positive semi-definite", i);
        TK_REQUIRE(std::isfinite(p->r[i]) && p->r[i] > 0.0, "r[%d] must be finite and > 0", i);
        TK_REQUIRE(!(p->lo[i] > p->hi[i]) && p->lo[i] == p->lo[i] && p->hi[i] == p->hi[i],
                   "clamp limits of coordinate %d are NaN or lo > hi", i);
        TK_REQUIRE(x0[i] >= p->lo[i] && x0[i] <= p->hi[i], "x0[%d] outside its clamp limits", i);
        k.x[i] = x0[i];
        k.v[i] = 0.0;
        k.pxx[i] = p->p0_pos[i];
        k.pxv[i] = 0.0;
        k.pvv[i] = p->p0_vel[i];
        k.qpp[i] = qpp;
        k.qpv[i] = qpv;
        k.qvv[i] = qvv;
        k.r[i] = p->r[i];
        k.lo[i] = p->lo[i];
        k.hi[i] = p->hi[i];
    }
    hipLaunchKernelGGL(kf_init_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s), k,
                       static_cast<KfState*>(d_kf));
    return check_launch("tk_kf_init");
}

tk_status tk_kf_step(void* d_kf, int32_t n, const double* d_z, double* d_theta, double* d_theta_next,
                     tk_stream s) {
    clear_error();
    TK_REQUIRE(n >= 1 && n <= kKfMax, "n = %d outside 1..%d", n, kKfMax);
    TK_REQUIRE(d_kf && d_z, "kf / z is NULL");
    hipLaunchKernelGGL(kf_step_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s),
                       static_cast<KfState*>(d_kf), n, d_z, d_theta, d_theta_next);
    return check_launch("tk_kf_step");
}

tk_status tk_cmaes_estimate(const void* d_state, int32_t n, int32_t lambda, const tk_chain* chains,
                            int32_t n_arms, double* d_z, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_state && d_z, "state / z is NULL");
    TK_REQUIRE(n_arms >= 1 && n_arms <= kMaxArms, "n_arms = %d outside 1..%d", n_arms, kMaxArms);
    TK_REQUIRE(n == 9 * n_arms, "n = %d must be 9 * n_arms = %d", n, 9 * n_arms);
    TK_REQUIRE(tk_cmaes_state_bytes(n, lambda) > 0, "invalid n = %d / lambda = %d", n, lambda);
    TK_REQUIRE(chains != nullptr, "chains is NULL");
    EstimateArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = n;
    a.lambda = lambda;
    for (int arm = 0; arm < n_arms; arm++)
        for (int j = 0; j < 3; j++) {
            const double lb = chains[arm].q_lb[j], ub = chains[arm].q_ub[j];
            TK_REQUIRE(std::isfinite(lb) && std::isfinite(ub) && ub > lb, "chain %d: joint %d has q_ub <= q_lb",
                       arm, j);
            a.lb[9 * arm + 6 + j] = lb;
            a.ub[9 * arm + 6 + j] = ub;
        }
    hipLaunchKernelGGL(cmaes_estimate_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s), d_state, a,
                       d_z);
    return check_launch("tk_cmaes_estimate");
}

}  // extern "C"
