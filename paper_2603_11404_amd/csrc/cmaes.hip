// CMA-ES sampling and update in FP64 (paper Sec. III-A.1, Eq. expected_fitness
// and Eq. cmaes_update; block-diagonal covariance of Sec. III-B).  Where the
// paper leaves the rules open (step size, evolution paths, h_sigma, default
// learning rates) the update follows Hansen's CMA-ES tutorial
// (arXiv:1604.00772).  Random numbers: Philox4x32-10 (Salmon et al., SC'11)
// keyed by the seed with counter (group j, candidate k, generation g, 0),
// mapped to normals by Box-Muller.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fitness_device.h"
#include "sample_device.h"

namespace tk {
namespace {

// ---------------------------------------------------------------- init

struct InitArgs {
    double mean0[kMaxN], offset[kMaxN], scale[kMaxN];
    double sigma0, c_m_scale, c_mu_scale, c1_scale;
    uint64_t seed;
    int32_t n, lambda, n_blocks;
    // offset from a device estimate in the filter's coordinates (when est is
    // set): coordinates in joint_mask are joint angles, encoded by the inverse
    // cosine map with limits lb/ub; those in reading_mask keep offset[]
    const double* est;
    double lb[kMaxN], ub[kMaxN];
    uint32_t joint_mask, reading_mask;
};

// Inverse cosine map (Sec. III-A.3): a joint angle q, clamped to [lb, ub], to
// the unconstrained coordinate in [lb, ub].
__device__ __forceinline__ double encode_joint(double q, double lb, double ub) {
    q = fmin(fmax(q, lb), ub);
    const double c = fmin(fmax(1.0 - 2.0 * (q - lb) / (ub - lb), -1.0), 1.0);
    return lb + (ub - lb) / kPi * acos(c);
}

__global__ __launch_bounds__(256) void cmaes_init_kernel(void* blob, InitArgs a) {
    StateView S = state_view(blob, a.n, a.lambda);
    const int n = a.n, lam = a.lambda, mu = lam / 2;
    const int tid = threadIdx.x;
    __shared__ double s_w[kMaxLambda];
    for (int i = tid; i < lam; i += blockDim.x)
        s_w[i] = i < mu ? log((lam + 1) / 2.0) - log(double(i + 1)) : 0.0;
    __syncthreads();
    if (tid == 0) {
        double sw = 0.0;
        for (int i = 0; i < mu; i++) sw += s_w[i];
        double sw2 = 0.0;
        for (int i = 0; i < mu; i++) {
            s_w[i] /= sw;
            sw2 += s_w[i] * s_w[i];
        }
        const double mu_eff = 1.0 / sw2;
        const double dn = n;
        const double c_sigma = (mu_eff + 2.0) / (dn + mu_eff + 5.0);
        const double d_sigma = 1.0 + 2.0 * fmax(0.0, sqrt((mu_eff - 1.0) / (dn + 1.0)) - 1.0) + c_sigma;
        const double c_c = (4.0 + mu_eff / dn) / (dn + 4.0 + 2.0 * mu_eff / dn);
        double c1 = 2.0 / ((dn + 1.3) * (dn + 1.3) + mu_eff);
        double c_mu = fmin(1.0 - c1, 2.0 * (mu_eff - 2.0 + 1.0 / mu_eff) / ((dn + 2.0) * (dn + 2.0) + mu_eff));
        c1 *= a.c1_scale;
        c_mu = fmin(c_mu * a.c_mu_scale, 1.0 - c1);
        *S.sigma = a.sigma0;
        *S.c_sigma = c_sigma;
        *S.d_sigma = d_sigma;
        *S.c_c = c_c;
        *S.c1 = c1;
        *S.c_mu = c_mu;
        *S.c_m = a.c_m_scale;
        *S.mu_eff = mu_eff;
        *S.chi_n = sqrt(dn) * (1.0 - 1.0 / (4.0 * dn) + 1.0 / (21.0 * dn * dn));
        *S.h_sigma = 1.0;
        S.hdr->gen = 0;
        S.hdr->seed = a.seed;
        S.hdr->flags = 0;
        S.hdr->magic = kStateMagic;
        S.hdr->n = n;
        S.hdr->lambda = lam;
        S.hdr->mu = mu;
        S.hdr->n_blocks = a.n_blocks;
        S.hdr->denom_gen = -1;
        S.hdr->denom = 0.0;
        S.hdr->z_gen = -1;
    }
    __syncthreads();
    for (int i = tid; i < lam; i += blockDim.x) {
        S.weights[i] = s_w[i];
        S.order[i] = i;
    }
    for (int i = tid; i < n; i += blockDim.x) {
        S.mean[i] = a.mean0[i];
        double off = a.offset[i];
        if (a.est != nullptr && !((a.reading_mask >> i) & 1u))
            off = ((a.joint_mask >> i) & 1u) ? encode_joint(a.est[i], a.lb[i], a.ub[i]) : a.est[i];
        S.offset[i] = off;
        S.scale[i] = a.scale[i];
        S.p_sigma[i] = 0.0;
        S.p_c[i] = 0.0;
        S.D[i] = 1.0;
    }
    for (int i = tid; i < n * n; i += blockDim.x) {
        const double v = (i / n == i % n) ? 1.0 : 0.0;
        S.C[i] = v;
        S.B[i] = v;
        S.L[i] = v;
    }
    for (int i = tid; i < lam * n; i += blockDim.x) {
        S.Z[i] = 0.0;
        S.Y[i] = 0.0;
    }
}

struct MeanArgs { double mean[kMaxN]; int32_t n, lambda; };

__global__ void cmaes_set_mean_kernel(void* blob, MeanArgs a) {
    StateView S = state_view(blob, a.n, a.lambda);
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) S.mean[i] = a.mean[i];
}

// ---------------------------------------------------------------- sample

// A 64-thread workgroup samples kSampCand candidates: first one thread per
// (candidate, group of four dimensions) draws z with Philox + Box-Muller, then
// one thread per (candidate, dimension) forms y = L z, x = m + sigma y and
// theta = offset + scale * x.
constexpr int kSampCand = 8;

__global__ __launch_bounds__(64) void cmaes_sample_kernel(void* blob, int n, int lam, float* __restrict__ X) {
    __shared__ double s_z[kSampCand][kMaxN + 3];
    __shared__ double s_Lf[kMaxN * kMaxN];   // the sampling factor L
    StateView S = state_view(blob, n, lam);
    const int tid = threadIdx.x;
    const int k0 = blockIdx.x * kSampCand;
    const uint32_t gen = uint32_t(S.hdr->gen);
    const uint64_t seed = S.hdr->seed;
    const uint32_t key0 = uint32_t(seed), key1 = uint32_t(seed >> 32);
    const int groups = (n + 3) / 4;
    for (int e = tid; e < n * n; e += 64) s_Lf[e] = S.L[e];
    for (int task = tid; task < kSampCand * groups; task += 64) {
        const int kk = task / groups, j = task % groups, k = k0 + kk;
        if (k >= lam) continue;
        draw_normals(key0, key1, gen, k, j, &s_z[kk][4 * j]);
    }
    __syncthreads();
    const double sigma = *S.sigma;
    for (int task = tid; task < kSampCand * n; task += 64) {
        const int kk = task / n, i = task % n, k = k0 + kk;
        if (k >= lam) continue;
        double y;
        X[k * n + i] = candidate_coord(s_Lf, s_z[kk], n, i, S.mean[i], sigma, S.offset[i], S.scale[i], &y);
        S.Z[k * n + i] = s_z[kk][i];
        S.Y[k * n + i] = y;
    }
    if (blockIdx.x == 0 && tid == 0) S.hdr->z_gen = int64_t(gen);   // Z: this generation's draws once all blocks end
}

// ---------------------------------------------------------------- update

constexpr int kWave64 = 64;
constexpr int kMaxSweeps = 30;
constexpr double kRotTol2 = 1e-26;      // Jacobi rotation threshold on a_pq^2 / |a_pp a_qq|
static_assert(kMaxSweeps % 2 == 0, "the Jacobi rounds run in pairs");

// Orders this wave's LDS writes before its later LDS reads (single-wave phases).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The rotations below use the hardware FP64 reciprocal square root (relative
// error at most about 5e-8) refined by Newton steps r <- r (1.5 - 0.5 x r^2)
// (explicit fused multiply-adds, the same in every form of the path): one step
// for sqrt(d^2 + 4 a_pq^2), which only sets the angle, and two for the
// normalisation, so that c and s are orthogonal to working precision, at a
// fraction of the latency of the correctly rounded square root and division.
// (Without the first step the iteration took about one round more.)
// The symmetric Schur rotation of the pair (p, q) = (2P, 2P+1), from its 2x2
// diagonal block: J(p, p) = J(q, q) = c, J(q, p) = s'_p = -s, J(p, q) =
// s'_q = +s, where tan(theta) = t zeroes the (p, q) entry of J^T A J:
//   t = 2 a_pq sign(d) / (|d| + sqrt(d^2 + 4 a_pq^2)),  d = a_qq - a_pp.
// Written without a division: with w = |d| + sqrt(d^2 + 4 a_pq^2),
// c = w / sqrt(w^2 + 4 a_pq^2) and s = 2 a_pq sign(d) / sqrt(w^2 + 4 a_pq^2).
// The pair is rotated only when a_pq^2 > kRotTol2 |a_pp a_qq|, i.e. when
// |a_pq| exceeds 1e-13 sqrt(|a_pp a_qq|); otherwise (c, s) = (1, 0).  A
// smaller threshold only polishes entries already far below what the
// conjugate path and the reconstruction B D^2 B^T = C resolve (about a round
// more on average at n = 9).
__device__ __forceinline__ bool pair_rotation(double app, double aqq, double apq, bool paired, double* c_out,
                                              double* sn_out) {
    const double d = aqq - app;
    const double p2 = apq * apq;
    const double q = 4.0 * p2;
    const double x = fma(d, d, q);
    const double hx = -0.5 * x;
    double r = __builtin_amdgcn_rsq(x);
    r = r * fma(hx * r, r, 1.5);
    const double w = fma(x, r, fabs(d));
    const double y = fma(w, w, q);
    const double hy = -0.5 * y;
    double t = __builtin_amdgcn_rsq(y);
    t = t * fma(hy * t, t, 1.5);
    t = t * fma(hy * t, t, 1.5);
    const double c = w * t;
    const double sn = (d >= 0.0 ? 2.0 * apq : -2.0 * apq) * t;
    const bool rot = paired && apq != 0.0 && p2 > kRotTol2 * fabs(app * aqq);
    *c_out = rot ? c : 1.0;
    *sn_out = rot ? sn : 0.0;
    return rot;
}

// The rotations of two pairs at once, each with exactly the arithmetic of
// pair_rotation.  The two chains are carried as the two elements of a vector
// and the steps are fenced against the instruction scheduler, so that the
// chains interleave in the wave's instruction stream instead of following one
// another (each step of one chain then fills the latency of the other's).
typedef double pair_f64 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ pair_f64 rsq2(pair_f64 v) {
    pair_f64 r;
    r.x = __builtin_amdgcn_rsq(v.x);
    r.y = __builtin_amdgcn_rsq(v.y);
    return r;
}

__device__ __forceinline__ void pair_rotation2(const double app_[2], const double aqq_[2], const double apq_[2],
                                               double c_out[2], double sn_out[2], bool rot_out[2]) {
    const pair_f64 app = {app_[0], app_[1]}, aqq = {aqq_[0], aqq_[1]}, apq = {apq_[0], apq_[1]};
    const pair_f64 one_half = {1.5, 1.5};
    const pair_f64 d = aqq - app;
    const pair_f64 p2 = apq * apq;
    // the rotation tests and the signs of s, off the chains
    bool rot[2];
    double sgn[2];
#pragma unroll
    for (int k = 0; k < 2; k++) {
        rot[k] = apq[k] != 0.0 && p2[k] > kRotTol2 * fabs(app[k] * aqq[k]);
        sgn[k] = d[k] >= 0.0 ? 2.0 * apq[k] : -2.0 * apq[k];
    }
    __builtin_amdgcn_sched_barrier(0);
    const pair_f64 q = 4.0 * p2;
    const pair_f64 x = __builtin_elementwise_fma(d, d, q);
    __builtin_amdgcn_sched_barrier(0);
    const pair_f64 hx = -0.5 * x;
    pair_f64 r = rsq2(x);
    __builtin_amdgcn_sched_barrier(0);
    r = r * __builtin_elementwise_fma(hx * r, r, one_half);
    __builtin_amdgcn_sched_barrier(0);
    const pair_f64 w = __builtin_elementwise_fma(x, r, __builtin_elementwise_abs(d));
    __builtin_amdgcn_sched_barrier(0);
    const pair_f64 y = __builtin_elementwise_fma(w, w, q);
    const pair_f64 hy = -0.5 * y;
    __builtin_amdgcn_sched_barrier(0);
    pair_f64 t = rsq2(y);
    __builtin_amdgcn_sched_barrier(0);
    t = t * __builtin_elementwise_fma(hy * t, t, one_half);
    __builtin_amdgcn_sched_barrier(0);
    t = t * __builtin_elementwise_fma(hy * t, t, one_half);
    __builtin_amdgcn_sched_barrier(0);
    const pair_f64 c = w * t;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        c_out[k] = rot[k] ? c[k] : 1.0;
        sn_out[k] = rot[k] ? sgn[k] * t[k] : 0.0;
        rot_out[k] = rot[k];
    }
}

// Quotient of small non-negative integers (a < 2^13, 1 <= b <= 2^10): an FP32
// reciprocal estimate within one of the quotient, then an exact integer
// correction each way (checked exhaustively over that range).
__device__ __forceinline__ int div_small(int a, int b) {
    int q = int(float(a) * __builtin_amdgcn_rcpf(float(b)));
    q += (q + 1) * b <= a ? 1 : 0;
    q -= q * b > a ? 1 : 0;
    return q;
}

// Row i of entry e of the upper triangle of an m x m matrix stored row by row
// (row i holds m - i entries, starting at i m - i (i - 1) / 2): the root of
// the quadratic as an estimate, then an exact correction each way.
__device__ __forceinline__ int tri_row(int e, int m) {
    const float b = float(2 * m + 1);
    int i = int(0.5f * (b - sqrtf(fmaxf(b * b - 8.0f * float(e), 0.0f))));
    auto start = [m](int r) { return r * m - (r * (r - 1)) / 2; };
    i += (i + 1 < m && start(i + 1) <= e) ? 1 : 0;
    i -= (i > 0 && start(i) > e) ? 1 : 0;
    return i;
}

// ---- ranking by (loss, index): a 64-element bitonic sort in the registers of
// one wave, then every element counts the elements ordered before it in the
// other waves' sorted lists by binary search.  The order is a total order (no
// two candidates share an index), so the result is the unique rank.

// The ranking compares 64-bit integers: a loss maps to an integer whose
// unsigned order is the order of the doubles (sign bit flipped for
// non-negative values, every bit for negative ones), after -0 is made +0 and
// NaN +inf, so that equal losses give equal integers.
__device__ __forceinline__ uint64_t order_key(double v) {
    v = (v != v) ? INFINITY : v + 0.0;
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
    return b ^ ((b >> 63) ? ~0ull : (1ull << 63));
}

// (key, index) record of a sorted list in LDS, read as one 16-byte word.
struct __align__(16) RankRec {
    uint64_t key;
    int32_t idx, pad;
};

// (ka, ia) ordered before (kb, ib), evaluated without branches.
__device__ __forceinline__ bool ordered_before(uint64_t ka, int ia, uint64_t kb, int ib) {
    return (ka < kb) | ((ka == kb) & (ia < ib));
}

// The value that lane (lane ^ S) holds, for S = 1 ... 32, without LDS: DPP
// quad permutations for 1 and 2, row rotations for 4 and 8 (rotating a
// 16-lane row by 8 is the exchange with lane ^ 8; by 4 and by 12 it reaches
// lane ^ 4 for lanes with bit 2 set and clear), the gfx950 16- and 32-lane
// swaps for 16 and 32.
template <int S>
__device__ __forceinline__ int lane_xor(int v, int lane) {
    if constexpr (S == 1) {
        return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);
    } else if constexpr (S == 2) {
        return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);
    } else if constexpr (S == 4) {
        const int a = __builtin_amdgcn_mov_dpp(v, 0x124, 0xF, 0xF, false);
        const int b = __builtin_amdgcn_mov_dpp(v, 0x12C, 0xF, 0xF, false);
        return (lane & 4) ? a : b;
    } else if constexpr (S == 8) {
        return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);
    } else if constexpr (S == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? int(r[0]) : int(r[1]);
    } else {
        static_assert(S == 32, "lane exchange distance");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? int(r[0]) : int(r[1]);
    }
}

template <int S>
__device__ __forceinline__ double lane_xor_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const uint32_t lo = uint32_t(lane_xor<S>(int(uint32_t(b)), lane));
    const uint32_t hi = uint32_t(lane_xor<S>(int(uint32_t(uint64_t(b) >> 32)), lane));
    return __longlong_as_double(static_cast<long long>((uint64_t(hi) << 32) | lo));
}

// Maximum over the wave (of values that are not NaN).
__device__ __forceinline__ double wave_max_f64(double v, int lane) {
    v = fmax(v, lane_xor_f64<32>(v, lane));
    v = fmax(v, lane_xor_f64<16>(v, lane));
    v = fmax(v, lane_xor_f64<8>(v, lane));
    v = fmax(v, lane_xor_f64<4>(v, lane));
    v = fmax(v, lane_xor_f64<2>(v, lane));
    return fmax(v, lane_xor_f64<1>(v, lane));
}

// One compare-exchange stage of the bitonic network: lanes lane and
// lane ^ STRIDE compare their (key, index); within blocks of SIZE lanes that
// sort ascending (bit SIZE of the lane clear) the lower lane keeps the first
// of the two, in descending blocks the second.
template <int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_stage(uint64_t& key, int& idx, int lane) {
    const uint32_t plo = uint32_t(lane_xor<STRIDE>(int(uint32_t(key)), lane));
    const uint32_t phi = uint32_t(lane_xor<STRIDE>(int(uint32_t(key >> 32)), lane));
    const uint64_t pk = (uint64_t(phi) << 32) | plo;
    const int pi = lane_xor<STRIDE>(idx, lane);
    const bool flip = ((lane & STRIDE) != 0) != ((lane & SIZE) != 0);
    const bool keep = ordered_before(key, idx, pk, pi) != flip;
    key = keep ? key : pk;
    idx = keep ? idx : pi;
}

template <int SIZE, int STRIDE>
__device__ __forceinline__ void bitonic_merge(uint64_t& key, int& idx, int lane) {
    bitonic_stage<SIZE, STRIDE>(key, idx, lane);
    if constexpr (STRIDE > 1) bitonic_merge<SIZE, STRIDE / 2>(key, idx, lane);
}

// Sorts the wave's 64 (key, index) pairs ascending: lane l ends with the l-th.
template <int SIZE = 64>
__device__ __forceinline__ void wave_sort64(uint64_t& key, int& idx, int lane) {
    if constexpr (SIZE > 2) wave_sort64<SIZE / 2>(key, idx, lane);
    bitonic_merge<SIZE, SIZE / 2>(key, idx, lane);
}

// Number of records of each of four sorted 64-record lists ordered before
// (key, idx): binary lifting over the answers 0 ... 64, the four searches
// advancing together so that their LDS reads overlap.
__device__ __forceinline__ void count_before64x4(const RankRec* const list[4], uint64_t key, int idx, int b[4]) {
#pragma unroll
    for (int q = 0; q < 4; q++) b[q] = 0;
#pragma unroll
    for (int s = 64; s >= 1; s >>= 1) {
        RankRec e[4];
#pragma unroll
        for (int q = 0; q < 4; q++) e[q] = list[q][min(b[q] + s - 1, 63)];
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] += ((b[q] + s <= 64) & ordered_before(e[q].key, e[q].idx, key, idx)) ? s : 0;
    }
}

// Dynamic LDS of the update: the elite rows Y[mu][n].
inline size_t update_lds_bytes(int n, int lam) { return sizeof(double) * size_t(n) * size_t(lam / 2); }

// dynamic LDS: elite rows Y[mu][n].  The state is staged in LDS first so that
// no loop below waits on global memory; sums over the elites are split into
// fixed-order partial sums (deterministic).
constexpr int kParts = 8;   // partial sums per output element

// Inputs and outputs of the fused tell-ask form: the losses are composed from
// the counts (and keypoints) of the evaluated candidates, and after the update
// the next generation is sampled and its forward kinematics evaluated.
struct TellAskArgs {
    const int32_t* counts;        // [lambda][2]
    const int32_t* target_count;  // |M|
    const float* kp;              // nullable [lambda][n_arms][4][2]
    const float* kp_ref;          // nullable [n_arms][4][2]
    LossArgs la;
    double* loss;                 // nullable [lambda], the composed losses
    float* X;                     // [lambda][n] next candidates
    FkArgs fk;
    float* link_xf;               // [lambda][n_arms][4][12]
    float* kp_next;               // nullable [lambda][n_arms][4][2]
};

// One problem's tell step in a batched launch.
struct UpdateJob {
    void* state;
    int32_t n, lam;
    TellAskArgs ta;
};

// A barrier over a group of n_waves waves of the workgroup through LDS (the
// update's waves on SIMDs other than wave 0's synchronise so while wave 0 runs
// the eigendecomposition, which a workgroup barrier would wait for).  bar:
// arrivals, generation, and a flag set if a wait ever exceeded its bound
// (about 0.1 s; it then goes on, so the kernel always ends).
constexpr int kWaitBound = 1 << 22;
__device__ __forceinline__ void wave_group_barrier(int* bar, int n_waves) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & (kWave64 - 1)) == 0) {
        const int g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__hip_atomic_fetch_add(&bar[0], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == n_waves - 1) {
            __hip_atomic_store(&bar[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(&bar[1], g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            int spin = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == g) {
                if (++spin == kWaitBound) {
                    __hip_atomic_store(&bar[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Arrival at a wave_group_barrier phase without waiting for it: the wave's
// LDS writes are released to the waves that wait, and the last wave to
// arrive, waiting or not, opens the barrier.
__device__ __forceinline__ void wave_group_arrive(int* bar, int n_waves) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & (kWave64 - 1)) == 0) {
        const int g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__hip_atomic_fetch_add(&bar[0], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == n_waves - 1) {
            __hip_atomic_store(&bar[0], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(&bar[1], g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Covariance update of the upper-triangle entries e = tid0, tid0 + stride, ...
// (rank-one + rank-mu from the partial sums, symmetric, block-masked) into Cn.
__device__ __forceinline__ void covariance_entries(int tid0, int stride, int n, int nb, int ntri, double keep,
                                                   double c1, double cmu, double delta, const double* pc,
                                                   const double* C, const double* partc, double* Cn) {
    for (int e = tid0; e < ntri; e += stride) {
        const int i = tri_row(e, n), j = i + e - (i * n - (i * (i - 1)) / 2);
        double rmu = 0.0;
        for (int part = 0; part < kParts; part++) rmu += partc[part * ntri + e];
        const double cij = keep * C[i * n + j] + c1 * (pc[i] * pc[j] + delta * C[i * n + j]) + cmu * rmu;
        const double cji = keep * C[j * n + i] + c1 * (pc[j] * pc[i] + delta * C[j * n + i]) + cmu * rmu;
        double v = 0.5 * (cij + cji);
        if (i / nb != j / nb) v = 0.0;   // block-diagonal covariance
        Cn[i * n + j] = v;
        Cn[j * n + i] = v;
    }
}

// Lower Cholesky factor of each diagonal block of C (n x n) into L (n x n,
// zero elsewhere), by one wave, with A as working copy: column k of every block at once,
// L_kk = sqrt(max'(A_kk)), L_ik = A_ik / L_kk, then A_ij -= L_ik L_jk for
// i >= j > k.  A pivot not above 1e-20 max_i A_ii is replaced by that floor.
// Returns (in every lane) whether a pivot was floored.
template <int CS>
__device__ __forceinline__ bool wave_cholesky(const double* C, double* A, double* L, int n, int nb, int lane) {
    const int n_blocks = n / nb, ntri_b = nb * (nb + 1) / 2, n_l = n_blocks * ntri_b;
    double dmax = 0.0;
    for (int i = lane; i < n; i += kWave64) dmax = fmax(dmax, C[i * n + i]);
    dmax = wave_max_f64(dmax, lane);
    double floor_v = 1e-20 * dmax;
    if (!(floor_v > 0.0)) floor_v = 2.2250738585072014e-308;   // smallest normal double
    for (int e = lane; e < n * n; e += kWave64) {
        L[e] = 0.0;
        A[e] = C[e];
    }
    // lane slots: entry (i, j), i >= j, of block b (lower triangle, row by row)
    int gi[CS], gj[CS];
    bool ok[CS];
#pragma unroll
    for (int sl = 0; sl < CS; sl++) {
        const int e = min(lane + kWave64 * sl, n_l - 1);
        const int b = div_small(e, ntri_b), eb = e - b * ntri_b;
        // row i holds i + 1 entries, starting at i (i + 1) / 2
        int i = int(0.5f * (sqrtf(8.0f * float(eb) + 1.0f) - 1.0f));
        i += ((i + 1) * (i + 2) / 2 <= eb) ? 1 : 0;
        i -= (i * (i + 1) / 2 > eb) ? 1 : 0;
        gi[sl] = b * nb + i;
        gj[sl] = b * nb + (eb - i * (i + 1) / 2);
        ok[sl] = lane + kWave64 * sl < n_l;
    }
    wave_sync();
    bool floored = false;
    for (int k = 0; k < nb; k++) {
#pragma unroll
        for (int sl = 0; sl < CS; sl++) {
            const int bk = gj[sl] - gj[sl] % nb + k;    // column k of the slot's block
            if (ok[sl] && gj[sl] == bk) {
                double piv = A[bk * n + bk];
                const bool fl = !(piv > floor_v);
                piv = fl ? floor_v : piv;
                const double lkk = sqrt(piv);
                L[gi[sl] * n + bk] = gi[sl] == bk ? lkk : A[gi[sl] * n + bk] / lkk;
                floored |= fl && gi[sl] == bk;
            }
        }
        wave_sync();
#pragma unroll
        for (int sl = 0; sl < CS; sl++) {
            const int bk = gj[sl] - gj[sl] % nb + k;
            if (ok[sl] && gj[sl] > bk)
                A[gi[sl] * n + gj[sl]] -= L[gi[sl] * n + bk] * L[gj[sl] * n + bk];
        }
        wave_sync();
    }
    return __ballot(floored) != 0ull;
}

// The update of one problem (Sec. III-A.1, Eq. (3)-(4), completed by Hansen's
// tutorial), in one workgroup.  The candidates were drawn as y = L z with
// L L^T = C; the conjugate path whitens with C^(-1/2) = B D^(-1) B^T from the
// eigendecomposition of that same C.  So wave 0 starts the eigendecomposition
// (Jacobi, warm-started from the previous B) as soon as the kernel starts,
// while the waves on the other SIMDs rank the candidates, recombine, form the
// rank-mu sums and, assuming h_sigma = 1, the new covariance and its Cholesky
// factor.  The two parts meet for the conjugate path; when h_sigma turns out
// 0 the covariance and factor are formed again with it.
//
// AS / VS: Jacobi entries per lane (upper-triangle / all within-block entries
// over 64 lanes); NT: threads of the workgroup; COMPOSE: losses composed from
// counts (tell); ASK: the next generation drawn at the end (tell-ask).
template <int AS, int VS, int NT, bool COMPOSE, bool ASK>
__device__ __forceinline__ void update_body(void* blob, const int n, const int lam, const double* __restrict__ loss,
                                            const TellAskArgs& ta) {
    extern __shared__ double s_elite[];  // [mu][n]
    __shared__ RankRec s_rec[kMaxLambda];   // the sorted lists of 64
    __shared__ double s_w[kMaxLambda / 2];
    // the eigendecomposition (wave 0): Jacobi buffers, the C the candidates
    // were drawn with, the previous eigenvectors, C B, the result
    __shared__ __align__(16) double s_A[kMaxN * kMaxN];
    __shared__ __align__(16) double s_T[kMaxN * kMaxN];
    __shared__ __align__(16) double s_V[kMaxN * kMaxN];
    __shared__ __align__(16) double s_Vn[kMaxN * kMaxN];
    __shared__ double s_Ce[kMaxN * kMaxN];
    __shared__ double s_Bw[kMaxN * kMaxN];
    __shared__ double s_X[kMaxN * kMaxN];
    __shared__ double s_B[kMaxN * kMaxN];
    __shared__ double s_D[kMaxN];
    __shared__ int s_pos[kMaxN];             // final Jacobi position of each index
    __shared__ int s_vsel;                   // the V buffer that holds the result
    __shared__ double s_sink[2 * kWave64];   // target of the V stores of lanes with no V entry
    // the other waves: C, the new covariance and its factor
    __shared__ double s_C[kMaxN * kMaxN];
    __shared__ double s_Cn[kMaxN * kMaxN];
    __shared__ double s_Cw[kMaxN * kMaxN];   // working copy of the factorisation
    __shared__ double s_L[kMaxN * kMaxN];
    __shared__ double s_part[kParts * kMaxN];                     // recombination partial sums
    __shared__ double s_partc[kParts * kMaxN * (kMaxN + 1) / 2];  // rank-mu partial sums
    __shared__ double s_yw[kMaxN], s_t[kMaxN], s_pc[kMaxN], s_pc1[kMaxN], s_ps[kMaxN], s_mean[kMaxN];
    __shared__ double s_scal[4];
    __shared__ int s_wbar[5];                // worker barrier: arrivals, generation, wait bound hit; y_w ready; V final
    __shared__ int s_zctr;                   // next z-draw task (chunks of 64 claimed by whole waves)
    __shared__ int s_flag[2];                // [0] eigenvalue floored, [1] Cholesky pivot floored / emax not finite

    StateView S = state_view(blob, n, lam);
    const int tid = threadIdx.x;
    const int lane = tid & (kWave64 - 1), wave = tid / kWave64;
    const int mu = S.hdr->mu;
    const int n_blocks = S.hdr->n_blocks;
    const int nb = n / n_blocks;
    const int nn = n * n;
    const int ntri = n * (n + 1) / 2;
    constexpr int NW = NT / kWave64;
    constexpr int NWW = NW - NW / 4;            // worker waves: w mod 4 != 0
    constexpr int NWK = NWW * kWave64;          // worker lanes
    constexpr int R = (kMaxLambda + NWK - 1) / NWK;   // candidates per worker lane
    constexpr int NMAX = AS == 1 ? 9 : kMaxN;   // n of the variant (n <= 9 uses AS = 1)
    constexpr bool kDrawZ = NMAX <= 9;          // the next generation's z drawn here
    constexpr int CS = (NMAX * (NMAX + 1) / 2 + kWave64 - 1) / kWave64;   // Cholesky entries per lane
    static_assert(NT >= 4 * kWave64, "wave 0 and three worker waves at least");
    const bool worker = (wave & 3) != 0;
    const int wi = wave - 1 - wave / 4;         // worker wave index (workers only)
    const int wk = wi * kWave64 + lane;         // worker lane index

    const double sigma = *S.sigma, c_m = *S.c_m, mu_eff = *S.mu_eff, cs = *S.c_sigma, cc = *S.c_c;
    const double c1 = *S.c1, cmu = *S.c_mu, chi_n = *S.chi_n, ds = *S.d_sigma;
    const int64_t gen = S.hdr->gen;
    // the h_sigma denominator of this generation when the previous update
    // cached it (same expression, same bits)
    const int64_t denom_gen = S.hdr->denom_gen;
    const double denom_cached = S.hdr->denom;
    // wave 0: C and the previous eigenvectors (the warm start of the
    // eigendecomposition) from the state, in flight across the barrier below:
    //   n <= 9: in the operand layouts of the FP64 16x16x4 matrix instruction,
    //   for the four k-steps s (lane (g, q) = (lane / 16, lane % 16) holds
    //   C(q, 4s + g) and B(4s + g, q), zero outside n x n);
    //   otherwise: row-major NMAX x NMAX, GE entries per lane.
    constexpr bool kMfmaWarm = NMAX <= 16;
    constexpr int GE = kMfmaWarm ? 4 : (NMAX * NMAX + kWave64 - 1) / kWave64;
    double cr[GE], br[GE];
    if (wave == 0) {
#pragma unroll
        for (int g = 0; g < GE; g++) {
            int i, j;
            bool in;
            if constexpr (kMfmaWarm) {
                i = 4 * g + (lane >> 4);
                j = lane & 15;
                in = i < n && j < n;
            } else {
                const int e = lane + g * kWave64;
                i = e / NMAX;
                j = e % NMAX;
                in = e < NMAX * NMAX && i < n && j < n;
            }
            const int ij = min(i, n - 1) * n + min(j, n - 1);   // in bounds; C is symmetric
            const double c = S.C[ij], b = S.B[ij];
            cr[g] = in ? c : 0.0;
            br[g] = in ? b : 0.0;
        }
    }
    if (tid == 0) {
        s_wbar[0] = 0;
        s_wbar[1] = 0;
        s_wbar[2] = 0;
        s_wbar[3] = 0;
        s_wbar[4] = 0;
        s_zctr = 0;
        s_flag[0] = 0;
        s_flag[1] = 0;
    }
    __syncthreads();

    // ---------------------------------------------------------- eigendecomposition (wave 0)
    const int m = nb + (nb & 1);
    const int k1 = m - 1;                      // rounds per sweep
    const int mm = m * m;
    const int ntri_m = m * (m + 1) / 2;
    const int n_a = n_blocks * ntri_m;         // upper-triangle entries of the blocks
    const int n_v = n_blocks * nb * m;         // V entries of the blocks
    auto move = [m](int p) {                   // position of an index in the next round
        if (m == 2 || p == 0) return p;
        if (p == 2) return 1;
        if (p & 1) return p + 2 <= m - 1 ? p + 2 : m - 2;
        return p - 2;
    };
    // (n <= 9) the next generation's z, exactly as a sampler would draw them
    // (they depend on the seed and generation only): one Philox block per
    // task, tasks in block-major order (so that a chunk holds one block index
    // j and the last block's unused normals are not computed), in chunks of
    // 64 tasks claimed by whole waves from an LDS counter.  The three waves
    // that share SIMD 0 with the eigendecomposition take chunks from the
    // start at the lowest priority, which leaves that wave's dependent chain
    // the issue slots; worker wave 0 joins after the Cholesky factor, worker
    // wave 1 only until V and D are final (it gathers B then), the other
    // workers after the covariance.  With up to 18 dimensions the draws would
    // outlast the eigendecomposition; the next generation's draw (ask-eval
    // prologue, sampler, or the tell-ask tail) makes them then.
    auto draw_z = [&](bool until_v_final) {
        const uint32_t gnext = uint32_t(gen + 1);
        const uint64_t seed = S.hdr->seed;
        const uint32_t key0 = uint32_t(seed), key1 = uint32_t(seed >> 32);
        const int n_tasks = lam * ((n + 3) / 4);
        for (;;) {
            if (until_v_final && __hip_atomic_load(&s_wbar[4], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
                break;
            int base = 0;
            if (lane == 0) base = __hip_atomic_fetch_add(&s_zctr, kWave64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            base = __builtin_amdgcn_readfirstlane(base);
            if (base >= n_tasks) break;
            const int task = base + lane;
            if (task < n_tasks) {
                const int j = div_small(task, lam), k = task - j * lam;
                double z[4];
                const int cnt = min(4, n - 4 * j);
                draw_normals_first(key0, key1, gnext, k, j, cnt, z);
                for (int t = 0; t < cnt; t++) S.Z[k * n + 4 * j + t] = z[t];
            }
        }
    };
    if (wave == 0) {
        __builtin_amdgcn_s_setprio(3);            // ahead of the drawing waves on this SIMD
        constexpr int kASlots = AS;
        static_assert(VS == 2 * AS, "two V entries per A entry");
        const int na_slots = (n_a + kWave64 - 1) / kWave64;
        // A lane holds the entry (i, j), i <= j, of block b of A, and two V
        // entries, in columns i and j: row j - i of column i and row
        // m - j + i of column j (when < nb), which covers rows 0..m of every
        // column exactly once over a block's entries.  What it reads comes in
        // aligned pairs of adjacent columns (c & ~1, c | 1) of one row, at
        // fixed offsets (in doubles, all even since m is even): rows i and
        // i^1 at columns j&~1 (its entry and the partner entries), rows i,
        // i^1 at i&~1 and rows j, j^1 at j&~1 (the operands of the two
        // rotations), and the two V rows at i&~1 and j&~1; it writes its
        // entry (mirrored) and its V entries at their next positions.
        int a_rij[kASlots], a_rpj[kASlots], a_li[kASlots], a_lj[kASlots];
        int a_w1[kASlots], a_w2[kASlots];
        int a_dp[kASlots], a_dq[kASlots];      // diagonal blocks of the pairs of positions i and j
        int v0_r[kASlots], v0_w[kASlots], v1_r[kASlots], v1_w[kASlots];
        bool a_ok[kASlots], a_off[kASlots], a_ei[kASlots], a_ej[kASlots], v0_ok[kASlots], v1_ok[kASlots];
#pragma unroll
        for (int sl = 0; sl < kASlots; sl++) {
            const int e = min(lane + kWave64 * sl, n_a - 1);
            const int b = div_small(e, ntri_m), eb = e - b * ntri_m;
            const int i = tri_row(eb, m);
            const int j = i + eb - (i * m - (i * (i - 1)) / 2), base = b * mm, vbase = b * nb * m;
            const int ie = i & ~1, je = j & ~1;
            a_rij[sl] = base + ie * m + je;           // rows 2P, 2P+1 of the entry's 2x2 block
            a_rpj[sl] = base + (ie + 1) * m + je;
            a_li[sl] = b * m + i;               // the lanes holding the rotations of positions i and j
            a_lj[sl] = b * m + j;
            a_dp[sl] = base + ie * m + ie;
            a_dq[sl] = base + je * m + je;
            a_w1[sl] = base + move(i) * m + move(j);
            a_w2[sl] = base + move(j) * m + move(i);
            a_ok[sl] = lane + kWave64 * sl < n_a;
            a_off[sl] = a_ok[sl] && i != j;
            a_ei[sl] = (i & 1) == 0;
            a_ej[sl] = (j & 1) == 0;
            const int r0 = j - i, r1 = m - j + i;
            v0_ok[sl] = a_ok[sl] && r0 < nb;
            v1_ok[sl] = a_ok[sl] && r1 < nb;
            v0_r[sl] = vbase + min(r0, nb - 1) * m + ie;
            v0_w[sl] = vbase + min(r0, nb - 1) * m + move(i);
            v1_r[sl] = vbase + min(r1, nb - 1) * m + je;
            v1_w[sl] = vbase + min(r1, nb - 1) * m + move(j);
        }
        // warm start: A = B^T C B (nearly diagonal when C changed little), V = B;
        // every rotation applies A <- J^T A J and V <- V J, so C = V diag(A) V^T at the end
        if constexpr (kMfmaWarm) {
            // X = C B and A' = B^T X on the matrix cores, n x n padded to 16 x 16.
            // The product's register r holds row g + 4r of column q, so X's
            // register s is exactly the second product's B operand at k-step s,
            // and B(4s + g, q) its A operand (B^T at (q, 4s + g)).
            typedef double f64x4 __attribute__((ext_vector_type(4)));
            f64x4 X = {0.0, 0.0, 0.0, 0.0}, Ap = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int st = 0; st < 4; st++) X = __builtin_amdgcn_mfma_f64_16x16x4f64(cr[st], br[st], X, 0, 0, 0);
#pragma unroll
            for (int st = 0; st < 4; st++) Ap = __builtin_amdgcn_mfma_f64_16x16x4f64(br[st], X[st], Ap, 0, 0, 0);
            // A' and V = B straight into the positional layouts (index l of
            // block b starts at position l); A' is symmetric up to rounding, and
            // the first round writes its rotated entries mirrored
            const int g = lane >> 4, q = lane & 15;
            const int bq = div_small(min(q, n - 1), nb);
#pragma unroll
            for (int st = 0; st < 4; st++) {
                const int row = g + 4 * st;               // A'(row, q) in register st; B(row, q) in br[st]
                if (row < n && q < n && div_small(row, nb) == bq) {
                    const int r = row - bq * nb, c = q - bq * nb;
                    s_A[bq * mm + r * m + c] = Ap[st];
                    s_V[bq * nb * m + r * m + c] = br[st];
                }
            }
            if (m > nb && lane < n_blocks * m) {
                // the dummy index of odd blocks: zero row and column of A, zero column of V
                const int b = div_small(lane, m), i = lane - b * m;
                s_A[b * mm + nb * m + i] = 0.0;
                s_A[b * mm + i * m + nb] = 0.0;
                if (i < nb) s_V[b * nb * m + i * m + nb] = 0.0;
            }
        } else {
            // in LDS as NMAX x NMAX matrices padded with zeros, so that the
            // products run over a fixed count (the padding adds exact zeros
            // after the terms of the sums)
#pragma unroll
            for (int g = 0; g < GE; g++) {
                const int e = lane + g * kWave64;
                if (e < NMAX * NMAX) {
                    s_Ce[e] = cr[g];
                    s_Bw[e] = br[g];
                }
            }
            wave_sync();
            for (int e = lane; e < NMAX * NMAX; e += kWave64) {
                const int i = e / NMAX, j = e % NMAX;
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < NMAX; k++) t += s_Ce[i * NMAX + k] * s_Bw[k * NMAX + j];
                s_X[e] = t;                                   // C B
            }
            for (int e = lane; e < n_v; e += kWave64) {
                // V = B in the positional layout: index l of block b starts at position l
                const int b = div_small(e, nb * m), rr = e - b * nb * m, r = div_small(rr, m), j = rr - r * m;
                s_V[e] = j < nb ? s_Bw[(b * nb + r) * NMAX + b * nb + j] : 0.0;
            }
            wave_sync();
            // A = B^T C B in the positional layout, symmetrised: 0.5 (A_ij + A_ji)
            // from both products (each summed over k in order); dummy rows and columns zero
            for (int e = lane; e < n_blocks * mm; e += kWave64) {
                const int b = div_small(e, mm), r = e - b * mm, i = div_small(r, m), j = r - i * m;
                const int gi = b * nb + min(i, nb - 1), gj = b * nb + min(j, nb - 1);
                double tij = 0.0, tji = 0.0;
#pragma unroll
                for (int k = 0; k < NMAX; k++) {
                    tij += s_Bw[k * NMAX + gi] * s_X[k * NMAX + gj];
                    tji += s_Bw[k * NMAX + gj] * s_X[k * NMAX + gi];
                }
                s_A[e] = (i < nb && j < nb) ? 0.5 * (tij + tji) : 0.0;
            }
        }
        wave_sync();
        {
            // Cyclic Jacobi in tournament order with a fixed pairing, run by wave 0
            // alone.  Each block is held in m = nb + (nb odd) positions (an odd
            // block gets a zero dummy index, which never rotates): A as an m x m
            // matrix and V as nb rows x m position columns.  In every round the
            // pairs are the positions (2k, 2k+1); after the round, indices move to
            // new positions (0 stays, 1 -> 3, 2 -> 1, other even p -> p - 2, other
            // odd p -> p + 2, the last odd position -> m - 2), a round-robin in
            // which every two indices of a block meet once per m - 1 rounds and the
            // layout returns to the start.  The rotated A and V are written straight
            // into their next positions, so every lane reads and writes the same LDS
            // addresses in every round and computes them once.  Per round:
            //   - the rotations of the pairs holding positions i and j of the lane's
            //     entry (i, j), from the pairs' 2x2 diagonal blocks: computed in the
            //     lane itself (one entry per lane) or taken from the lane of each
            //     position by cross-lane shuffles (several);
            //   - the entry of A' = J^T A J (mirrored) and two entries of V' = V J,
            //     written into the other buffer at the next round's positions (with
            //     no rotation this only moves the indices);
            //   - when nothing rotated, the test whether any pair exceeds the
            //     rotation threshold; if none does, the iteration has converged
            //     (another sweep would rotate nothing).
            const int max_rounds = kMaxSweeps * k1;   // even (kMaxSweeps is)
            // constants of the conjugate path and the step size, ahead of need
            const double ps_gain = sqrt(cs * (2.0 - cs) * mu_eff);
            const double denom = denom_gen == gen ? denom_cached : sqrt(1.0 - pow(1.0 - cs, 2.0 * double(gen + 1)));
            const double h_bound = (1.4 + 2.0 / (n + 1.0)) * chi_n;
            const double cs_ds = cs / ds;
            int moved = 0;                             // rounds applied (index moves) modulo k1
            // (several entries per lane) lane t < n_blocks m computes the rotation
            // of the pair holding position t, from the pair's 2x2 diagonal block
            // (rows 2P, 2P+1 at column 2P)
            const int n_pos = n_blocks * m;
            const int t_pos = min(tid, n_pos - 1);
            const int t_b = div_small(t_pos, m), t_p = t_pos - t_b * m, t_2P = t_p & ~1;
            const int t_rp = t_b * mm + t_2P * m + t_2P, t_rq = t_rp + m;
            const bool t_even = (t_p & 1) == 0;
            auto pair = [](const double* base, int off) { return *reinterpret_cast<const double2*>(base + off); };
            // One round from (Ac, Vc) into (An, Vn); true when it found the
            // iteration converged.  Every round rotates and moves the indices (with
            // no rotation this only moves them); the test whether to stop follows
            // the stores, so that it is not on the path from one round to the next.
            auto jacobi_round = [&](const double* Ac, double* An, const double* Vc, double* Vn) -> bool {
                // the entry's 2x2 block B (rows 2P, 2P+1, columns 2Q, 2Q+1) and the
                // two V rows at columns 2P and 2Q, read with no branch (every slot's
                // offsets are valid; slots past the last entry repeat it)
                double2 blk0[kASlots], blk1[kASlots], vr0[kASlots], vr1[kASlots];
                auto read_blocks = [&]() {
        #pragma unroll
                    for (int sl = 0; sl < kASlots; sl++) {
                        blk0[sl] = pair(Ac, a_rij[sl]);
                        blk1[sl] = pair(Ac, a_rpj[sl]);
                        vr0[sl] = pair(Vc, v0_r[sl]);
                        vr1[sl] = pair(Vc, v1_r[sl]);
                    }
                };
                // the rotation columns u, w of positions i and j, and A(i, i), A(j, j)
                double u0[kASlots], u1[kASlots], w0[kASlots], w1[kASlots], di[kASlots], dj[kASlots];
                bool rot;
                if constexpr (AS == 1) {
                    // one entry per lane: the lane computes both rotations itself
                    // from the pairs' diagonal blocks (read with its other operands),
                    // with no exchange between lanes
                    const double2 p0 = pair(Ac, a_dp[0]), p1 = pair(Ac, a_dp[0] + m);
                    const double2 q0 = pair(Ac, a_dq[0]), q1 = pair(Ac, a_dq[0] + m);
                    read_blocks();   // issued behind the diagonal blocks, consumed after the rotations
                    const double app[2] = {p0.x, q0.x}, aqq[2] = {p1.y, q1.y}, apq[2] = {p0.y, q0.y};
                    double cs2[2], sn2[2];
                    bool r2[2];
                    pair_rotation2(app, aqq, apq, cs2, sn2, r2);
                    const double cp = cs2[0], sp = sn2[0], cq = cs2[1], sq = sn2[1];
                    const bool rp = r2[0], rq = r2[1];
                    // column of the pair rotation: (c, -s) at an even position, (s, c) at an odd one
                    u0[0] = a_ei[0] ? cp : sp;
                    u1[0] = a_ei[0] ? -sp : cp;
                    w0[0] = a_ej[0] ? cq : sq;
                    w1[0] = a_ej[0] ? -sq : cq;
                    di[0] = a_ei[0] ? p0.x : p1.y;
                    dj[0] = a_ej[0] ? q0.x : q1.y;
                    rot = rp || rq;
                } else {
                    // lane t < n_blocks m computes the rotation of the pair holding
                    // position t; the entry lanes take the columns by cross-lane shuffles
                    const double2 bp = pair(Ac, t_rp), bq = pair(Ac, t_rq);
                    read_blocks();
                    double c_t, sn_t;
                    rot = pair_rotation(bp.x, bq.y, bp.y, tid < n_pos, &c_t, &sn_t);
                    const double dd_t = t_even ? bp.x : bq.y;       // A(t, t)
                    const double col0_t = t_even ? c_t : sn_t, col1_t = t_even ? -sn_t : c_t;
        #pragma unroll
                    for (int sl = 0; sl < kASlots; sl++) {
                        u0[sl] = __shfl(col0_t, a_li[sl]);
                        u1[sl] = __shfl(col1_t, a_li[sl]);
                        w0[sl] = __shfl(col0_t, a_lj[sl]);
                        w1[sl] = __shfl(col1_t, a_lj[sl]);
                        di[sl] = __shfl(dd_t, a_li[sl]);
                        dj[sl] = __shfl(dd_t, a_lj[sl]);
                    }
                }
        #pragma unroll
                for (int sl = 0; sl < kASlots; sl++) {
                    if (sl == 0 || sl < na_slots) {   // slot 0 always holds an entry (n >= 1)
                        // A'(i, j) = u^T B w; a lane past the last entry recomputes the
                        // last entry, so its duplicate stores write the same value
                        const double r0 = fma(w0[sl], blk0[sl].x, w1[sl] * blk0[sl].y);
                        const double r1 = fma(w0[sl], blk1[sl].x, w1[sl] * blk1[sl].y);
                        const double v = fma(u0[sl], r0, u1[sl] * r1);
                        An[a_w1[sl]] = v;
                        An[a_w2[sl]] = v;
                        // V'(r, i) = V(r, 2P) u0 + V(r, 2P+1) u1, likewise at column j
                        double* d0 = v0_ok[sl] ? Vn + v0_w[sl] : s_sink + tid;
                        double* d1 = v1_ok[sl] ? Vn + v1_w[sl] : s_sink + kWave64 + tid;
                        *d0 = fma(u0[sl], vr0[sl].x, u1[sl] * vr0[sl].y);
                        *d1 = fma(w0[sl], vr1[sl].x, w1[sl] * vr1[sl].y);
                    }
                }
                wave_sync();
                moved = moved + 1 == k1 ? 0 : moved + 1;
                if (__ballot(rot) != 0ull) return false;
                // nothing rotated in this round: converged when no pair exceeds the
                // threshold (another sweep would rotate nothing)
                bool open = false;
        #pragma unroll
                for (int sl = 0; sl < kASlots; sl++) {
                    if (sl == 0 || sl < na_slots) {   // slot 0 always holds an entry (n >= 1)
                        const double2 row = a_ei[sl] ? blk0[sl] : blk1[sl];
                        const double aij = a_ej[sl] ? row.x : row.y;
                        open |= a_off[sl] && aij * aij > kRotTol2 * fabs(di[sl] * dj[sl]);
                    }
                }
                return __ballot(open) == 0ull;
            };
            // the rounds alternate between two buffer pairs; the result is in the
            // pair the last round wrote
            const double* Acur = s_A;
            const double* Vcur = s_V;
            for (int it = 0; it < max_rounds; it += 2) {
                if (jacobi_round(s_A, s_T, s_V, s_Vn)) {
                    Acur = s_T;
                    Vcur = s_Vn;
                    break;
                }
                if (jacobi_round(s_T, s_A, s_Vn, s_V)) break;
            }
            // final position of every index; D = sqrt(eigenvalues) with a floor
            // at 1e-20 * max (the maximum over the lanes ignores NaN like a
            // running fmax from 0).  B is V with its columns in index order,
            // gathered after the workgroup barrier below; the conjugate path
            // reads V through the positions.
            if (lane == 0) s_vsel = Vcur == s_V ? 0 : 1;
            // The moves keep position 0 and cycle the others through
            // 1, 3, 5, ..., m - 1, m - 2, ..., 4, 2 (index c: odd p at
            // (p - 1) / 2, even p at m - 1 - p / 2), so after `moved` rounds the
            // index that started at p sits at cycle index (c + moved) mod (m - 1).
            double ev = 0.0;
            int pos_l = 0;
            const int lb = lane < n ? div_small(lane, nb) : 0;     // block of index `lane`
            const int l_row = lane < n ? lane - lb * nb : 0;       // its row within the block
            if (l_row != 0) {
                int c = ((l_row & 1) ? (l_row - 1) / 2 : m - 1 - l_row / 2) + moved;
                c -= c >= k1 ? k1 : 0;
                pos_l = c < m / 2 ? 2 * c + 1 : 2 * (m - 1 - c);
            }
            if (lane < n) s_pos[lane] = pos_l;
            // the V entries of the conjugate path, read now (this wave's own
            // data): column pos_l of the lane's block for B^T y_w, and row l_row
            // at the positions of the block's indices for B t (the position of
            // index j of a block is the same in every block: lane j's)
            const double* Vb = Vcur + lb * nb * m;
            double vcol[NMAX], vrow[NMAX];
#pragma unroll
            for (int i = 0; i < NMAX; i++) {
                const int ic = min(i, nb - 1);
                const int pos_i = __builtin_amdgcn_readlane(pos_l, ic);
                vcol[i] = Vb[ic * m + pos_l];
                vrow[i] = Vb[l_row * m + pos_i];
            }
            ev = Acur[lb * mm + pos_l * m + pos_l];
            const double emax = wave_max_f64(lane < n ? fmax(0.0, ev) : 0.0, lane);
            const double floor_v = 1e-20 * emax;
            const bool floored = lane < n && !(ev >= floor_v);
            const double d_l = sqrt(floored ? floor_v : ev);
            if (lane < n) s_D[lane] = d_l;
            if (lane == 0) s_flag[0] = (__ballot(floored) != 0ull ? 1 : 0) | (emax < INFINITY ? 0 : 2);
            // V, the positions and D are final: a worker wave gathers B
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) __hip_atomic_store(&s_wbar[4], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            // 5. the conjugate path p_sigma with C^(-1/2) y_w = B D^(-1) B^T y_w
            //    (y_w from the first worker wave, long done by now), its length,
            //    h_sigma and sigma
            if (lane == 0) {
                int spin = 0;
                while (__hip_atomic_load(&s_wbar[3], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
                    if (++spin == kWaitBound) {
                        __hip_atomic_store(&s_wbar[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            // (B^T y_w)_l = sum_i V(i, pos l) y_w,i over the rows i of l's block;
            // (B t)_l = sum_j V(l, pos j) t_j over the indices j of l's block (the
            // other blocks' terms of the full sums are exact zeros)
            double t_l = 0.0;
            if (lane < n) {
                double acc = 0.0;
    #pragma unroll
                for (int i = 0; i < NMAX; i++)
                    if (i < nb) acc += vcol[i] * s_yw[lb * nb + i];
                t_l = acc / d_l;
            }
            double bt = 0.0;
            if (n_blocks == 1) {
                // one block: t_j is lane j's value, read with readlane (no LDS round trip)
                const uint64_t tb = static_cast<uint64_t>(__double_as_longlong(t_l));
                const int t_lo = int(uint32_t(tb)), t_hi = int(uint32_t(tb >> 32));
    #pragma unroll
                for (int j = 0; j < NMAX; j++) {
                    if (j < nb) {
                        const uint64_t w = (uint64_t(uint32_t(__builtin_amdgcn_readlane(t_hi, j))) << 32) |
                                           uint32_t(__builtin_amdgcn_readlane(t_lo, j));
                        bt += vrow[j] * __longlong_as_double(static_cast<long long>(w));
                    }
                }
            } else {
                if (lane < n) s_t[lane] = t_l;
                wave_sync();
    #pragma unroll
                for (int j = 0; j < NMAX; j++)
                    if (j < nb) bt += vrow[j] * s_t[lb * nb + j];
            }
            double ps_l = 0.0;
            if (lane < n) {
                ps_l = (1.0 - cs) * s_ps[lane] + ps_gain * bt;
                S.p_sigma[lane] = ps_l;
            }
            // ||p_sigma||^2 by a fixed butterfly over the lanes
            double ss = ps_l * ps_l;
            ss += lane_xor_f64<32>(ss, lane);
            ss += lane_xor_f64<16>(ss, lane);
            ss += lane_xor_f64<8>(ss, lane);
            ss += lane_xor_f64<4>(ss, lane);
            ss += lane_xor_f64<2>(ss, lane);
            ss += lane_xor_f64<1>(ss, lane);
            if (lane == 0) {
                const double ps_norm = sqrt(ss);
                s_scal[0] = ps_norm;
                s_scal[1] = (ps_norm / denom < h_bound) ? 1.0 : 0.0;
                const double sg = sigma * exp(cs_ds * (ps_norm / chi_n - 1.0));
                s_scal[3] = sg;
                if (!(sg > 0.0 && sg < INFINITY)) s_flag[0] |= 2;
                // (every read of the old p_sigma and sigma precedes the y_w flag)
                *S.h_sigma = s_scal[1];
                *S.sigma = sg;
            }
        }
    } else if (worker) {
        // ------------------------------------------------------ ranking and the covariance (waves on other SIMDs)
        // 0. Worker lane wk holds candidates k = wk + r NWK (r < R), i.e. entry
        //    `lane` of list l = wi + r NWW of 64 candidates, with their keys
        //    and rows of Y; keys past lambda are +inf, and their indices order
        //    them last.  The state goes through registers into LDS after the
        //    sort, so that its loads and the count loads are in flight together.
        uint64_t kr[R];
        int ir[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int k = wk + r * NWK;
            double v = INFINITY;
            if (k < lam) {
                if (COMPOSE) {
                    v = compose_loss_one(ta.counts[2 * k], ta.counts[2 * k + 1], *ta.target_count,
                                         ta.kp ? ta.kp + size_t(k) * ta.la.n_arms * 8 : nullptr, ta.kp_ref, ta.la);
                    if (ta.loss) ta.loss[k] = v;
                } else {
                    v = loss[k];
                }
            }
            kr[r] = order_key(v);
            ir[r] = k;
        }
        double yr[R][NMAX];
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int k = wk + r * NWK;
#pragma unroll
            for (int i = 0; i < NMAX; i++) yr[r][i] = (k < lam && i < n) ? S.Y[size_t(k) * n + i] : 0.0;
        }
        // 1a. each worker wave sorts its lists of 64 (key, index) pairs in
        //     registers (NaN ranks as +inf) and stores them in LDS
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int l = wi + r * NWW;
            if (64 * l < lam) {   // uniform over the wave
                wave_sort64(kr[r], ir[r], lane);
                s_rec[64 * l + lane] = RankRec{kr[r], ir[r], 0};
            }
        }
        for (int i = wk; i < mu; i += NWK) s_w[i] = S.weights[i];
        for (int e = wk; e < nn; e += NWK) s_C[e] = S.C[e];
        if (wk < n) {
            s_pc[wk] = S.p_c[wk];
            s_ps[wk] = S.p_sigma[wk];
            s_mean[wk] = S.mean[wk];
        }
        wave_group_barrier(s_wbar, NWW);

        // 1b. rank = position in the own sorted list + the number of records
        //     ordered before it in each other list (four searches side by
        //     side).  The rank goes back to the lane that holds the candidate's
        //     row of Y (a lane of the same wave), which writes the elite rows.
        const int n_lists = (lam + 63) / 64;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const int l = wi + r * NWW;
            if (64 * l < lam) {
                const int idx = ir[r];
                const uint64_t key = kr[r];
                int rank = lane;
                for (int l0 = 0; l0 < n_lists; l0 += 4) {   // uniform trip count
                    const RankRec* lists[4];
                    int b[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) lists[q] = s_rec + 64 * min(l0 + q, n_lists - 1);
                    count_before64x4(lists, key, idx, b);
#pragma unroll
                    for (int q = 0; q < 4; q++) rank += (l0 + q >= n_lists || l0 + q == l) ? 0 : b[q];
                }
                if (idx < lam) S.order[rank] = idx;
                // sorted lane -> the lane of candidate idx (idx mod 64): its rank
                const int my_rank = __builtin_amdgcn_ds_permute(4 * (idx & (kWave64 - 1)), rank);
                if (my_rank < mu && wk + r * NWK < lam) {
#pragma unroll
                    for (int i = 0; i < NMAX; i++)
                        if (i < n) s_elite[my_rank * n + i] = yr[r][i];
                }
            }
        }
        wave_group_barrier(s_wbar, NWW);

        // 2. weighted recombination y_w = sum_r w_r y_{r:lambda}: partial sums
        for (int task = wk; task < kParts * n; task += NWK) {
            const int part = task / n, i = task % n;
            double acc = 0.0;
#pragma unroll 4
            for (int r = part; r < mu; r += kParts) acc += s_w[r] * s_elite[r * n + i];
            s_part[part * n + i] = acc;
        }
        wave_group_barrier(s_wbar, NWW);

        // 3. (worker wave 0) y_w, the mean, and the evolution path p_c as it is
        //    when h_sigma = 1; (the others) the sum of the weights and the
        //    rank-mu partial sums of the upper triangle
        if (wi == 0) {
            if (lane < n) {
                double acc = 0.0;
                for (int part = 0; part < kParts; part++) acc += s_part[part * n + lane];
                s_yw[lane] = acc;
                const double mnew = s_mean[lane] + c_m * sigma * acc;
                s_mean[lane] = mnew;
                S.mean[lane] = mnew;
                s_pc1[lane] = (1.0 - cc) * s_pc[lane] + 1.0 * sqrt(cc * (2.0 - cc) * mu_eff) * acc;
            }
            // y_w is ready for the conjugate path (wave 0)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) __hip_atomic_store(&s_wbar[3], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            if (wi == 1) {
                // sum of the recombination weights: strided partial sums, then a fixed butterfly
                double sw = 0.0;
                for (int r = lane; r < mu; r += kWave64) sw += s_w[r];
                for (int off = kWave64 / 2; off > 0; off >>= 1) sw += __shfl_xor(sw, off);
                if (lane == 0) s_scal[2] = sw;
            }
            for (int task = wk - kWave64; task < kParts * ntri; task += NWK - kWave64) {
                const int part = task / ntri, e = task - part * ntri;
                const int i = tri_row(e, n), j = i + e - (i * n - (i * (i - 1)) / 2);
                double acc = 0.0;
#pragma unroll 4
                for (int r = part; r < mu; r += kParts) acc += s_w[r] * s_elite[r * n + i] * s_elite[r * n + j];
                s_partc[part * ntri + e] = acc;
            }
        }
        wave_group_barrier(s_wbar, NWW);

        // 4. the new covariance for h_sigma = 1 (rank-one term from that p_c,
        //    no h_sigma correction), then its Cholesky factor (worker wave 0)
        //    while the other workers draw the next generation's z
        covariance_entries(wk, NWK, n, nb, ntri, 1.0 - c1 - cmu * s_scal[2], c1, cmu, 0.0, s_pc1, s_C, s_partc,
                           s_Cn);
        // worker wave 0 (the factor) waits for every entry; the others go on at once
        if (wi == 0)
            wave_group_barrier(s_wbar, NWW);
        else
            wave_group_arrive(s_wbar, NWW);
        if (wi == 0) {
            const bool fl = wave_cholesky<CS>(s_Cn, s_Cw, s_L, n, nb, lane);
            if (lane == 0) s_flag[1] = fl ? 1 : 0;
            // the new C, its factor and p_c as they are when h_sigma = 1 (written
            // again below otherwise)
            if (lane < n) S.p_c[lane] = s_pc1[lane];
            for (int e = lane; e < nn; e += kWave64) {
                S.C[e] = s_Cn[e];
                S.L[e] = s_L[e];
            }
            if (kDrawZ) draw_z(false);
        } else {
            // the next generation's h_sigma denominator, cached in the state with
            // its generation
            if (wk == kWave64) {
                S.hdr->denom = sqrt(1.0 - pow(1.0 - cs, 2.0 * double(gen + 2)));
                S.hdr->denom_gen = gen + 1;
                if (kDrawZ) S.hdr->z_gen = gen + 1;   // every task of Z is claimed and written before the kernel ends
            }
            if (kDrawZ) draw_z(wi == 1);
            if (wi == 1) {
                // B = V with its columns in index order (position s_pos[j] holds
                // index j), and D, once wave 0 has them
                if (lane == 0) {
                    int spin = 0;
                    while (__hip_atomic_load(&s_wbar[4], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == 0) {
                        if (++spin == kWaitBound) {
                            __hip_atomic_store(&s_wbar[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                const double* Vres = s_vsel ? s_Vn : s_V;
                for (int e = lane; e < nn; e += kWave64) {
                    const int i = div_small(e, n), j = e - i * n, b = div_small(i, nb);
                    const double v = b == div_small(j, nb) ? Vres[b * nb * m + (i - b * nb) * m + s_pos[j]] : 0.0;
                    s_B[e] = v;
                    S.B[e] = v;
                }
                if (lane < n) S.D[lane] = s_D[lane];
                if (kDrawZ) draw_z(false);           // the draws left, if any
            }
        }
    } else if (kDrawZ) {
        draw_z(false);                            // the waves beside wave 0 on SIMD 0 (priority 0)
    }
    __syncthreads();
    const double h_sigma = s_scal[1];

    if (h_sigma != 1.0) {
        // h_sigma = 0: p_c without the y_w term, the covariance with the h_sigma
        // correction, and its factor again
        if (tid < n) s_pc1[tid] = (1.0 - cc) * s_pc[tid] + h_sigma * sqrt(cc * (2.0 - cc) * mu_eff) * s_yw[tid];
        __syncthreads();
        covariance_entries(tid, NT, n, nb, ntri, 1.0 - c1 - cmu * s_scal[2], c1, cmu, (1.0 - h_sigma) * cc * (2.0 - cc),
                           s_pc1, s_C, s_partc, s_Cn);
        __syncthreads();
        if (wave == 0) {
            const bool fl = wave_cholesky<CS>(s_Cn, s_Cw, s_L, n, nb, lane);
            if (lane == 0) s_flag[1] = fl ? 1 : 0;
        }
        __syncthreads();
        if (tid < n) S.p_c[tid] = s_pc1[tid];
        for (int e = tid; e < nn; e += NT) {
            S.C[e] = s_Cn[e];
            S.L[e] = s_L[e];
        }
    }
    // the rest of the state (p_sigma, sigma and h_sigma are written by wave 0):
    // generation, flags
    if (tid == 0) {
        S.hdr->gen = gen + 1;
        S.hdr->flags = ((s_flag[0] | s_flag[1]) & 1) | (s_flag[0] & 2) | (s_wbar[2] ? 4 : 0);
    }
    if (!ASK) return;

    // 6. (tell-ask form) the next generation: the same draws and arithmetic as
    //    the sample kernel (z by Philox + Box-Muller with the incremented
    //    generation, y = L z, x = m + sigma y, theta = offset + scale x), then
    //    the forward kinematics of every candidate and arm
    const double sigma_next = s_scal[3];
    if (!kDrawZ) {
        // the next generation's z (not drawn beside the eigendecomposition)
        const uint32_t gnext = uint32_t(gen + 1);
        const uint64_t seed = S.hdr->seed;
        const uint32_t key0 = uint32_t(seed), key1 = uint32_t(seed >> 32);
        const int groups = (n + 3) / 4;
        for (int task = tid; task < lam * groups; task += NT) {
            const int k = div_small(task, groups), j = task - k * groups;
            double z[4];
            draw_normals(key0, key1, gnext, k, j, z);
            for (int t = 0; t < 4; t++)
                if (4 * j + t < n) S.Z[k * n + 4 * j + t] = z[t];
        }
        if (tid == 0) S.hdr->z_gen = gen + 1;
        __syncthreads();
    }
    for (int task = tid; task < lam * n; task += NT) {
        const int k = task / n, i = task % n;
        double y;
        ta.X[task] = candidate_coord(s_L, S.Z + size_t(k) * n, n, i, s_mean[i], sigma_next, S.offset[i],
                                     S.scale[i], &y);
        S.Y[task] = y;
    }
    __syncthreads();
    for (int task = tid; task < lam * ta.fk.n_arms; task += NT) {
        const int arm = task % ta.fk.n_arms;
        const ChainK ch = arm == 0 ? ta.fk.ch[0] : ta.fk.ch[1];
        fk_candidate(ta.X + size_t(task) * 9, ch, ta.fk.cam, ta.link_xf + size_t(task) * 48,
                     ta.kp_next ? ta.kp_next + size_t(task) * 8 : nullptr);
    }
}


template <int AS, int VS, int NT, bool COMPOSE, bool ASK>
__global__ __launch_bounds__(NT) void cmaes_update_kernel(void* blob, int n, int lam, const double* __restrict__ loss,
                                                          TellAskArgs ta) {
    update_body<AS, VS, NT, COMPOSE, ASK>(blob, n, lam, loss, ta);
}

// Many problems in one launch: workgroup i runs the tell step (loss
// composition + update) of problem prob[i], described in device memory.
template <int AS, int VS, int NT>
__global__ __launch_bounds__(NT) void cmaes_tell_batch_kernel(const UpdateJob* __restrict__ table, BatchList L) {
    const UpdateJob& j = table[L.prob[blockIdx.x]];
    update_body<AS, VS, NT, true, false>(j.state, j.n, j.lam, nullptr, j.ta);
}
}  // namespace
}  // namespace tk

namespace tk {

static tk_status check_state(const void* d_state, int32_t n, int32_t lambda) {
    TK_REQUIRE(d_state != nullptr, "state is NULL");
    TK_REQUIRE((reinterpret_cast<uintptr_t>(d_state) & 255) == 0, "state must be 256-byte aligned");
    TK_REQUIRE(n >= 1 && n <= kMaxN, "n = %d outside 1..%d", n, kMaxN);
    TK_REQUIRE(lambda >= 2 && lambda <= kMaxLambda, "lambda = %d outside 2..%d", lambda, kMaxLambda);
    return TK_OK;
}

size_t batch_update_entry_bytes() { return sizeof(UpdateJob); }

tk_status batch_describe_update(const tk_problem& p, void* dst) {
    if (tk_status st = check_state(p.d_state, p.n, p.lambda)) return st;
    TK_REQUIRE(p.d_counts && p.d_target_count, "counts / target_count is NULL");
    UpdateJob j;
    std::memset(&j, 0, sizeof j);
    const float* kp = p.d_kp_ref ? p.d_kp : nullptr;
    if (tk_status st = make_loss_args(p.lambda, p.kind, p.lambda_app, kp, p.d_kp_ref, p.n_arms, p.lambda_kp, p.tau,
                                      &j.ta.la))
        return st;
    j.state = p.d_state;
    j.n = p.n;
    j.lam = p.lambda;
    j.ta.counts = p.d_counts;
    j.ta.target_count = p.d_target_count;
    j.ta.kp = kp;
    j.ta.kp_ref = p.d_kp_ref;
    j.ta.loss = p.d_loss;
    std::memcpy(dst, &j, sizeof j);
    return TK_OK;
}

// One launch per variant class (n <= 9 / n <= 18) and per kMaxBatch problems.
tk_status batch_launch_tell(const tk_problem* problems, int32_t n, const void* d_entries, hipStream_t s) {
    const UpdateJob* table = static_cast<const UpdateJob*>(d_entries);
    for (int large = 0; large < 2; large++) {
        BatchList L;
        std::memset(&L, 0, sizeof L);
        size_t lds = 0;
        auto flush = [&]() -> tk_status {
            if (L.count == 0) return TK_OK;
            if (large)
                hipLaunchKernelGGL((cmaes_tell_batch_kernel<3, 6, 512>), dim3(L.count), dim3(512), lds, s, table, L);
            else
                hipLaunchKernelGGL((cmaes_tell_batch_kernel<1, 2, 1024>), dim3(L.count), dim3(1024), lds, s, table, L);
            L.count = 0;
            lds = 0;
            return check_launch("tk_batch_tell");
        };
        for (int i = 0; i < n; i++) {
            if ((problems[i].n > 9) != bool(large)) continue;
            L.prob[L.count++] = i;
            lds = std::max(lds, update_lds_bytes(problems[i].n, problems[i].lambda));
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

size_t tk_cmaes_state_bytes(int32_t n, int32_t lambda) {
    if (n < 1 || n > kMaxN || lambda < 2 || lambda > kMaxLambda) return 0;
    tk_cmaes_layout L;
    cmaes_layout(n, lambda, &L);
    return size_t(L.total_bytes);
}

tk_status tk_cmaes_layout_get(int32_t n, int32_t lambda, tk_cmaes_layout* out) {
    clear_error();
    TK_REQUIRE(out != nullptr, "out is NULL");
    TK_REQUIRE(n >= 1 && n <= kMaxN, "n = %d outside 1..%d", n, kMaxN);
    TK_REQUIRE(lambda >= 2 && lambda <= kMaxLambda, "lambda = %d outside 2..%d", lambda, kMaxLambda);
    cmaes_layout(n, lambda, out);
    return TK_OK;
}


// The scalar settings shared by both initialisations.
static tk_status init_settings(InitArgs& a, int32_t n, int32_t lambda, double sigma0, const tk_cmaes_params* p,
                               uint64_t seed) {
    TK_REQUIRE(sigma0 > 0.0 && std::isfinite(sigma0), "sigma0 must be finite and > 0");
    a.sigma0 = sigma0;
    a.c_m_scale = p ? p->c_m_scale : 1.0;
    a.c_mu_scale = p ? p->c_mu_scale : 1.0;
    a.c1_scale = p ? p->c1_scale : 1.0;
    a.n_blocks = p ? p->n_blocks : 1;
    TK_REQUIRE(a.c_m_scale > 0 && a.c_mu_scale > 0 && a.c1_scale > 0, "learning-rate scales must be > 0");
    TK_REQUIRE(a.n_blocks >= 1 && n % a.n_blocks == 0, "n_blocks = %d must divide n = %d", a.n_blocks, n);
    a.seed = seed;
    a.n = n;
    a.lambda = lambda;
    return TK_OK;
}

tk_status tk_cmaes_init_at(void* d_state, int32_t n, int32_t lambda, const double* d_est, const tk_chain* chains,
                           int32_t n_arms, const double* readings, double sigma0, const double* scale,
                           const tk_cmaes_params* p, uint64_t seed, tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(d_est && chains && scale, "d_est / chains / scale is NULL");
    TK_REQUIRE(n_arms >= 1 && n_arms <= kMaxArms && n == 9 * n_arms, "n = %d must be 9 x n_arms (n_arms = %d)", n,
               n_arms);
    InitArgs a;
    std::memset(&a, 0, sizeof a);
    if (tk_status st = init_settings(a, n, lambda, sigma0, p, seed)) return st;
    a.est = d_est;
    for (int i = 0; i < n; i++) {
        TK_REQUIRE(std::isfinite(scale[i]), "non-finite scale[%d]", i);
        a.scale[i] = scale[i];
    }
    for (int arm = 0; arm < n_arms; arm++) {
        for (int j = 0; j < 3; j++) {
            const int i = 9 * arm + 6 + j;
            const double lb = chains[arm].q_lb[j], ub = chains[arm].q_ub[j];
            TK_REQUIRE(std::isfinite(lb) && std::isfinite(ub) && lb < ub, "arm %d joint %d: limits must satisfy lb < ub",
                       arm, j);
            a.lb[i] = lb;
            a.ub[i] = ub;
            a.joint_mask |= 1u << i;
            if (readings) {
                TK_REQUIRE(std::isfinite(readings[3 * arm + j]), "non-finite reading of arm %d joint %d", arm, j);
                a.offset[i] = readings[3 * arm + j];
                a.reading_mask |= 1u << i;
            }
        }
    }
    hipLaunchKernelGGL(cmaes_init_kernel, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(s), d_state, a);
    return check_launch("tk_cmaes_init_at");
}

tk_status tk_cmaes_init(void* d_state, int32_t n, int32_t lambda, const double* mean0, double sigma0,
                        const double* offset, const double* scale, const tk_cmaes_params* p, uint64_t seed,
                        tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(mean0 && offset && scale, "mean0/offset/scale must be host arrays of n doubles");
    InitArgs a;
    std::memset(&a, 0, sizeof a);
    if (tk_status st = init_settings(a, n, lambda, sigma0, p, seed)) return st;
    for (int i = 0; i < n; i++) {
        TK_REQUIRE(std::isfinite(mean0[i]) && std::isfinite(offset[i]) && std::isfinite(scale[i]),
                   "non-finite mean0/offset/scale[%d]", i);
        a.mean0[i] = mean0[i];
        a.offset[i] = offset[i];
        a.scale[i] = scale[i];
    }
    hipLaunchKernelGGL(cmaes_init_kernel, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(s), d_state, a);
    return check_launch("tk_cmaes_init");
}

tk_status tk_cmaes_set_mean(void* d_state, int32_t n, int32_t lambda, const double* mean, tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(mean != nullptr, "mean is NULL");
    MeanArgs a;
    std::memset(&a, 0, sizeof a);
    for (int i = 0; i < n; i++) {
        TK_REQUIRE(std::isfinite(mean[i]), "non-finite mean[%d]", i);
        a.mean[i] = mean[i];
    }
    a.n = n;
    a.lambda = lambda;
    hipLaunchKernelGGL(cmaes_set_mean_kernel, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(s), d_state, a);
    return check_launch("tk_cmaes_set_mean");
}

tk_status tk_cmaes_sample(void* d_state, int32_t n, int32_t lambda, float* d_X, tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(d_X != nullptr, "X is NULL");
    hipLaunchKernelGGL(cmaes_sample_kernel, dim3((lambda + kSampCand - 1) / kSampCand), dim3(64), 0,
                       reinterpret_cast<hipStream_t>(s), d_state, n, lambda, d_X);
    return check_launch("tk_cmaes_sample");
}

tk_status tk_cmaes_update(void* d_state, int32_t n, int32_t lambda, const double* d_loss, tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(d_loss != nullptr, "loss is NULL");
    const size_t lds = update_lds_bytes(n, lambda);
    // Jacobi entries inside the blocks number at most n(n+1)/2 (upper
    // triangle) and n^2 (all), whatever the block count: for n <= 9 they fit
    // one and two per lane of a wave, for n <= 18 three and six.
    TellAskArgs none;
    std::memset(&none, 0, sizeof none);
    if (n <= 9) {
        hipLaunchKernelGGL((cmaes_update_kernel<1, 2, 1024, false, false>), dim3(1), dim3(1024), lds,
                           reinterpret_cast<hipStream_t>(s), d_state, n, lambda, d_loss, none);
    } else {
        hipLaunchKernelGGL((cmaes_update_kernel<3, 6, 512, false, false>), dim3(1), dim3(512), lds,
                           reinterpret_cast<hipStream_t>(s), d_state, n, lambda, d_loss, none);
    }
    return check_launch("tk_cmaes_update");
}

tk_status tk_cmaes_tell(void* d_state, int32_t n, int32_t lambda, const int32_t* d_counts,
                        const int32_t* d_target_count, int32_t kind, double lambda_app, const float* d_kp,
                        const float* d_kp_ref, int32_t n_arms, double lambda_kp, double tau, double* d_loss,
                        tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(d_counts && d_target_count, "counts / target_count is NULL");
    TellAskArgs ta;
    std::memset(&ta, 0, sizeof ta);
    if (tk_status st = make_loss_args(lambda, kind, lambda_app, d_kp, d_kp_ref, n_arms, lambda_kp, tau, &ta.la))
        return st;
    ta.counts = d_counts;
    ta.target_count = d_target_count;
    ta.kp = d_kp;
    ta.kp_ref = d_kp_ref;
    ta.loss = d_loss;
    const size_t lds = update_lds_bytes(n, lambda);
    if (n <= 9) {
        hipLaunchKernelGGL((cmaes_update_kernel<1, 2, 1024, true, false>), dim3(1), dim3(1024), lds,
                           reinterpret_cast<hipStream_t>(s), d_state, n, lambda, nullptr, ta);
    } else {
        hipLaunchKernelGGL((cmaes_update_kernel<3, 6, 512, true, false>), dim3(1), dim3(512), lds,
                           reinterpret_cast<hipStream_t>(s), d_state, n, lambda, nullptr, ta);
    }
    return check_launch("tk_cmaes_tell");
}

tk_status tk_cmaes_tell_ask(void* d_state, int32_t n, int32_t lambda, const int32_t* d_counts,
                            const int32_t* d_target_count, int32_t kind, double lambda_app, const float* d_kp,
                            const float* d_kp_ref, double lambda_kp, double tau, double* d_loss,
                            const tk_chain* chains, int32_t n_arms, const tk_camera* cam, float* d_X,
                            float* d_link_xf, float* d_kp_next, tk_stream s) {
    clear_error();
    if (tk_status st = check_state(d_state, n, lambda)) return st;
    TK_REQUIRE(d_counts && d_target_count, "counts / target_count is NULL");
    TK_REQUIRE(d_X && d_link_xf, "X / link_xf is NULL");
    TellAskArgs ta;
    std::memset(&ta, 0, sizeof ta);
    if (tk_status st = make_loss_args(lambda, kind, lambda_app, d_kp, d_kp_ref, n_arms, lambda_kp, tau, &ta.la))
        return st;
    if (tk_status st = make_fk_args(chains, n_arms, cam, &ta.fk)) return st;
    TK_REQUIRE(n == 9 * n_arms, "n = %d must be 9 x n_arms = %d", n, 9 * n_arms);
    ta.fk.batch = lambda;
    ta.counts = d_counts;
    ta.target_count = d_target_count;
    ta.kp = d_kp;
    ta.kp_ref = d_kp_ref;
    ta.loss = d_loss;
    ta.X = d_X;
    ta.link_xf = d_link_xf;
    ta.kp_next = d_kp_next;
    const size_t lds = update_lds_bytes(n, lambda);
    if (n <= 9) {
        hipLaunchKernelGGL((cmaes_update_kernel<1, 2, 1024, true, true>), dim3(1), dim3(1024), lds,
                           reinterpret_cast<hipStream_t>(s), d_state, n, lambda, nullptr, ta);
    } else {
        hipLaunchKernelGGL((cmaes_update_kernel<3, 6, 512, true, true>), dim3(1), dim3(512), lds,
                           reinterpret_cast<hipStream_t>(s), d_state, n, lambda, nullptr, ta);
    }
    return check_launch("tk_cmaes_tell_ask");
}

}  // extern "C"
