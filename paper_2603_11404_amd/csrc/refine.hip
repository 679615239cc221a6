// Gradient refinement of the CMA-ES mean with Adam (Kingma and Ba), in the
// normalised space x of the search (theta = offset + scale x), on the
// gradient of the soft-silhouette loss.  The mean is read as an FP32
// candidate for the forward kinematics, and Adam steps move the FP64 mean of
// the state in place; the state's sigma, paths and covariance are untouched.
#include <cmath>
#include <cstring>

#include "fitness_device.h"

namespace tk {
namespace {

__global__ __launch_bounds__(64) void mean_candidate_kernel(const void* __restrict__ blob, int32_t n, int32_t lam,
                                                            float* __restrict__ X) {
    const int i = threadIdx.x;
    if (i >= n) return;
    StateView S = state_view(const_cast<void*>(blob), n, lam);
    X[i] = float(S.offset[i] + S.scale[i] * S.mean[i]);
}

struct AdamArgs {
    double lr, beta1, beta2, eps;
    int32_t n, lam;
};

// adam state: m[n], v[n], t (as a double) -- 8 (2n + 1) bytes
__global__ __launch_bounds__(64) void adam_kernel(void* __restrict__ blob, const float* __restrict__ grad_theta,
                                                  double* __restrict__ adam, AdamArgs a) {
    const int i = threadIdx.x;
    StateView S = state_view(blob, a.n, a.lam);
    const double t = adam[2 * a.n] + 1.0;
    if (i < a.n) {
        const double g = double(grad_theta[i]) * S.scale[i];   // d/dx = d/dtheta * scale
        const double m = a.beta1 * adam[i] + (1.0 - a.beta1) * g;
        const double v = a.beta2 * adam[a.n + i] + (1.0 - a.beta2) * g * g;
        adam[i] = m;
        adam[a.n + i] = v;
        const double mh = m / (1.0 - pow(a.beta1, t));
        const double vh = v / (1.0 - pow(a.beta2, t));
        S.mean[i] = S.mean[i] - a.lr * mh / (sqrt(vh) + a.eps);
    }
    __builtin_amdgcn_wave_barrier();
    if (i == 0) adam[2 * a.n] = t;
}

// One refinement step in one launch: the Adam step of adam_kernel (when a
// gradient is given), then the mean as an FP32 candidate and its forward
// kinematics (one lane per arm), the same arithmetic as mean_candidate_kernel
// and fk_kernel.
__global__ __launch_bounds__(64) void adam_transform_kernel(void* __restrict__ blob,
                                                            const float* __restrict__ grad_theta,
                                                            double* __restrict__ adam, AdamArgs a, FkArgs f,
                                                            float* __restrict__ X, float* __restrict__ link_xf) {
    __shared__ float s_x[9 * kMaxArms];
    const int i = threadIdx.x;
    StateView S = state_view(blob, a.n, a.lam);
    if (grad_theta != nullptr) {
        const double t = adam[2 * a.n] + 1.0;
        if (i < a.n) {
            const double g = double(grad_theta[i]) * S.scale[i];
            const double m = a.beta1 * adam[i] + (1.0 - a.beta1) * g;
            const double v = a.beta2 * adam[a.n + i] + (1.0 - a.beta2) * g * g;
            adam[i] = m;
            adam[a.n + i] = v;
            const double mh = m / (1.0 - pow(a.beta1, t));
            const double vh = v / (1.0 - pow(a.beta2, t));
            S.mean[i] = S.mean[i] - a.lr * mh / (sqrt(vh) + a.eps);
        }
        __builtin_amdgcn_wave_barrier();
        if (i == 0) adam[2 * a.n] = t;
    }
    if (i < a.n) {
        const float x = float(S.offset[i] + S.scale[i] * S.mean[i]);
        X[i] = x;
        s_x[i] = x;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (link_xf != nullptr && i < f.n_arms) {
        const ChainK ch = i == 0 ? f.ch[0] : f.ch[1];
        fk_candidate(s_x + 9 * i, ch, f.cam, link_xf + size_t(i) * 48, nullptr);
    }
}

__global__ __launch_bounds__(64) void adam_reset_kernel(double* __restrict__ adam, int32_t count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) adam[i] = 0.0;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_cmaes_mean_candidate(const void* d_state, int32_t n, int32_t lambda, float* d_X, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_state && d_X, "state / X is NULL");
    TK_REQUIRE(tk_cmaes_state_bytes(n, lambda) > 0, "invalid n = %d / lambda = %d", n, lambda);
    hipLaunchKernelGGL(mean_candidate_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s), d_state, n,
                       lambda, d_X);
    return check_launch("tk_cmaes_mean_candidate");
}

tk_status tk_adam_reset(void* d_adam, int32_t n, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_adam != nullptr, "adam state is NULL");
    TK_REQUIRE(n >= 1 && n <= kMaxN, "n = %d outside 1..%d", n, kMaxN);
    hipLaunchKernelGGL(adam_reset_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s),
                       static_cast<double*>(d_adam), 2 * n + 1);
    return check_launch("tk_adam_reset");
}

tk_status tk_cmaes_adam(void* d_state, int32_t n, int32_t lambda, const float* d_grad_theta, void* d_adam,
                        double lr, double beta1, double beta2, double eps, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_state && d_grad_theta && d_adam, "state / grad / adam state is NULL");
    TK_REQUIRE(tk_cmaes_state_bytes(n, lambda) > 0, "invalid n = %d / lambda = %d", n, lambda);
    TK_REQUIRE(std::isfinite(lr) && lr > 0.0, "lr must be finite and > 0");
    TK_REQUIRE(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0, "betas must lie in [0, 1)");
    TK_REQUIRE(std::isfinite(eps) && eps > 0.0, "eps must be finite and > 0");
    AdamArgs a{lr, beta1, beta2, eps, n, lambda};
    hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s), d_state, d_grad_theta,
                       static_cast<double*>(d_adam), a);
    return check_launch("tk_cmaes_adam");
}

tk_status tk_cmaes_adam_transform(void* d_state, int32_t n, int32_t lambda, const float* d_grad_theta,
                                  void* d_adam, double lr, double beta1, double beta2, double eps, int32_t n_arms,
                                  const tk_chain* chains, float* d_X, float* d_link_xf, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_state && d_X, "state / X is NULL");
    TK_REQUIRE(tk_cmaes_state_bytes(n, lambda) > 0, "invalid n = %d / lambda = %d", n, lambda);
    TK_REQUIRE(d_grad_theta == nullptr || d_adam != nullptr, "adam state is NULL");
    TK_REQUIRE(n == 9 * n_arms, "n = %d is not 9 x n_arms = %d", n, 9 * n_arms);
    TK_REQUIRE(std::isfinite(lr) && lr > 0.0, "lr must be finite and > 0");
    TK_REQUIRE(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0, "betas must lie in [0, 1)");
    TK_REQUIRE(std::isfinite(eps) && eps > 0.0, "eps must be finite and > 0");
    FkArgs f;
    if (tk_status st = make_fk_args(chains, n_arms, nullptr, &f)) return st;
    f.batch = 1;
    AdamArgs a{lr, beta1, beta2, eps, n, lambda};
    hipLaunchKernelGGL(adam_transform_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s), d_state,
                       d_grad_theta, static_cast<double*>(d_adam), a, f, d_X, d_link_xf);
    return check_launch("tk_cmaes_adam_transform");
}

}  // extern "C"
