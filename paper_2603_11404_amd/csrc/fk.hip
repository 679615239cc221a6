// Forward kinematics of the candidates and loss composition.
//
// FK (Sec. III-A.3): cosine joint map qhat -> q in [lb, ub]; look-at rotation
// R = Ry(gamma) Rx(alpha) Rz(beta) with translation (x, y, z) gives T_r^c; the
// link chain T_l(q) of the instrument gives M_l = T_r^c T_l, the transform
// applied to the mesh vertices of link l by the renderer
// S = R(K(Pi(T_r^c T_m^r(q) v_m))) of Sec. III-A.2.  One thread per
// (candidate, arm), FP32.
//
// Loss (Eq. (5), (6), (8); mask error 1 - IoU of Sec. IV): one thread per
// candidate, FP64 from integer counts.
#include <cmath>
#include <cstring>

#include "fitness_device.h"

namespace tk {
namespace {

__global__ __launch_bounds__(64) void fk_kernel(const float* __restrict__ X, FkArgs a, float* __restrict__ link_xf,
                                                float* __restrict__ kp) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= a.batch * a.n_arms) return;
    const int arm = idx % a.n_arms;
    const ChainK ch = arm == 0 ? a.ch[0] : a.ch[1];   // selected, not indexed: keeps the chain in registers
    fk_candidate(X + size_t(idx) * 9, ch, a.cam, link_xf + size_t(idx) * 48, kp ? kp + size_t(idx) * 8 : nullptr);
}

__global__ __launch_bounds__(256) void compose_loss_kernel(const int32_t* __restrict__ counts,
                                                           const int32_t* __restrict__ target_count,
                                                           const float* __restrict__ kp,
                                                           const float* __restrict__ kp_ref, LossArgs a,
                                                           double* __restrict__ loss) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.batch) return;
    loss[b] = compose_loss_one(counts[2 * b], counts[2 * b + 1], *target_count,
                               kp ? kp + size_t(b) * a.n_arms * 8 : nullptr, kp_ref, a);
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_fk_transform(const float* d_X, int32_t batch, int32_t n_arms, const tk_chain* chains, float* d_link_xf,
                          float* d_kp, const tk_camera* cam, tk_stream s) {
    clear_error();
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    TK_REQUIRE(batch == 0 || (d_X != nullptr && d_link_xf != nullptr), "X / link_xf is NULL");
    FkArgs a;
    if (tk_status st = make_fk_args(chains, n_arms, d_kp ? cam : nullptr, &a)) return st;
    a.batch = batch;
    if (batch == 0) return TK_OK;
    // 64-thread blocks: the work is a latency chain per thread, so spread it over CUs
    const int total = batch * n_arms, threads = 64;
    hipLaunchKernelGGL(fk_kernel, dim3((total + threads - 1) / threads), dim3(threads), 0,
                       reinterpret_cast<hipStream_t>(s), d_X, a, d_link_xf, d_kp);
    return check_launch("tk_fk_transform");
}

tk_status tk_compose_loss(const int32_t* d_counts, int32_t batch, const int32_t* d_target_count, int32_t kind,
                          double lambda_app, const float* d_kp, const float* d_kp_ref, int32_t n_arms,
                          double lambda_kp, double tau, double* d_loss, tk_stream s) {
    clear_error();
    TK_REQUIRE(batch >= 0, "batch = %d < 0", batch);
    TK_REQUIRE(batch == 0 || (d_counts && d_target_count && d_loss), "counts / target_count / loss is NULL");
    LossArgs a;
    if (tk_status st = make_loss_args(batch, kind, lambda_app, d_kp, d_kp_ref, n_arms, lambda_kp, tau, &a)) return st;
    if (batch == 0) return TK_OK;
    const int threads = 256;
    hipLaunchKernelGGL(compose_loss_kernel, dim3((batch + threads - 1) / threads), dim3(threads), 0,
                       reinterpret_cast<hipStream_t>(s), d_counts, d_target_count, d_kp, d_kp_ref, a, d_loss);
    return check_launch("tk_compose_loss");
}

}  // extern "C"
