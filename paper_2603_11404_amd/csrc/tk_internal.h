// Internal declarations shared by the HIP sources of libtk (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "tk.h"

namespace tk {

// ---------------------------------------------------------------- errors

void set_error(const std::string& msg);
void clear_error();
tk_status fail(tk_status s, const char* fmt, ...);
tk_status check_launch(const char* what);

#define TK_REQUIRE(cond, ...)                                            \
    do {                                                                 \
        if (!(cond)) return ::tk::fail(TK_ERR_INVALID_ARGUMENT, __VA_ARGS__); \
    } while (0)

// ---------------------------------------------------------------- limits

constexpr int kMaxN = 18;          // CMA-ES dimension (two arms x 9)
constexpr int kMaxLambda = 1024;   // population size
constexpr int kMaxArms = 2;
constexpr int kMaxImage = 4096;    // width / height limit
constexpr int kMaxBatch = 128;     // problems per batched launch
constexpr int kGuardQ8 = 32768 * 256;  // guard band in Q8 units

// ---------------------------------------------------------------- CMA-ES state layout

struct StateHeader {               // first 64 bytes of the blob
    int64_t gen;
    uint64_t seed;
    int32_t flags;
    int32_t magic;
    int32_t n, lambda, mu, n_blocks;
    int64_t denom_gen;             // generation g of the cached h_sigma denominator (-1: none)
    double denom;                  // sqrt(1 - (1 - c_sigma)^(2 (g + 1))) for g = denom_gen
    int64_t z_gen;                 // generation whose draws Z holds for every candidate (-1: none)
};
static_assert(sizeof(StateHeader) == 64, "state header is 64 bytes");
static_assert(offsetof(StateHeader, z_gen) == 56, "z_gen offset in the layout");
constexpr int32_t kStateMagic = 0x544b4345;  // "ECKT"

__host__ __device__ inline void cmaes_layout(int32_t n, int32_t lam, tk_cmaes_layout* L) {
    int64_t o = 0;
    L->gen = 0;
    L->seed = 8;
    L->flags = 16;
    L->z_gen = 56;
    o = 64;
    auto take = [&o](int64_t bytes) {
        int64_t r = o;
        o += (bytes + 7) & ~int64_t(7);
        return r;
    };
    L->sigma = take(8);
    L->c_sigma = take(8);
    L->d_sigma = take(8);
    L->c_c = take(8);
    L->c1 = take(8);
    L->c_mu = take(8);
    L->c_m = take(8);
    L->mu_eff = take(8);
    L->chi_n = take(8);
    L->h_sigma = take(8);
    L->weights = take(8 * int64_t(lam));
    L->mean = take(8 * int64_t(n));
    L->p_sigma = take(8 * int64_t(n));
    L->p_c = take(8 * int64_t(n));
    L->offset = take(8 * int64_t(n));
    L->scale = take(8 * int64_t(n));
    L->D = take(8 * int64_t(n));
    L->C = take(8 * int64_t(n) * n);
    L->B = take(8 * int64_t(n) * n);
    L->Z = take(8 * int64_t(lam) * n);
    L->Y = take(8 * int64_t(lam) * n);
    L->order = take(4 * int64_t(lam));
    L->L = take(8 * int64_t(n) * n);
    L->total_bytes = (o + 255) & ~int64_t(255);
}

// Typed view of a state blob.
struct StateView {
    StateHeader* hdr;
    double *sigma, *c_sigma, *d_sigma, *c_c, *c1, *c_mu, *c_m, *mu_eff, *chi_n, *h_sigma;
    double *weights, *mean, *p_sigma, *p_c, *offset, *scale, *D, *C, *B, *Z, *Y, *L;
    int32_t* order;
};

__host__ __device__ inline StateView state_view(void* blob, int32_t n, int32_t lam) {
    tk_cmaes_layout L;
    cmaes_layout(n, lam, &L);
    char* b = static_cast<char*>(blob);
    StateView v;
    v.hdr = reinterpret_cast<StateHeader*>(b);
#define TK_F(f) v.f = reinterpret_cast<double*>(b + L.f)
    TK_F(sigma); TK_F(c_sigma); TK_F(d_sigma); TK_F(c_c); TK_F(c1); TK_F(c_mu); TK_F(c_m);
    TK_F(mu_eff); TK_F(chi_n); TK_F(h_sigma); TK_F(weights); TK_F(mean); TK_F(p_sigma);
    TK_F(p_c); TK_F(offset); TK_F(scale); TK_F(D); TK_F(C); TK_F(B); TK_F(Z); TK_F(Y); TK_F(L);
#undef TK_F
    v.order = reinterpret_cast<int32_t*>(b + L.order);
    return v;
}

// ---------------------------------------------------------------- geometry structs passed to kernels

struct CamK {                     // camera as seen by the kernels
    float fx, fy, cx, cy, z_near;
    int32_t width, height, words_x, words_y;
};

inline CamK make_cam(const tk_camera& c) {
    CamK k;
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy; k.z_near = c.z_near;
    k.width = c.width; k.height = c.height;
    k.words_x = (c.width + 7) / 8;
    k.words_y = (c.height + 7) / 8;
    return k;
}

struct MeshK {
    const float* vertices;
    const int32_t* triangles;
    const uint8_t* vertex_link;
    int32_t n_vertices, n_triangles, vertex_offset;  // offset into concatenated snapped arrays
    int32_t closed;                                  // tk_mesh.closed
};

struct MeshSet {
    MeshK m[kMaxArms];
    int32_t n_meshes;
    int32_t total_vertices;
};

// Kinematic chain as the kernels see it (FP32).
struct ChainK {
    float d, lb[3], ub[3], kp[4][3];
    int32_t kp_link[4];
};

struct FkArgs {
    ChainK ch[kMaxArms];
    CamK cam;
    int32_t batch, n_arms;
};

// Weights of the loss composition.
struct LossArgs {
    double lambda_app, lambda_kp, tau;
    int32_t batch, kind, n_arms;
};

// Problem list of a batched launch (kernel argument).
struct BatchList {
    int32_t count;
    int32_t prob[kMaxBatch];
};

// Batched problems: each problem's device descriptors (one raster entry, one
// update entry) are written into a host table by the describe functions and
// read by the batched kernels from the caller's device copy.
size_t batch_raster_entry_bytes();
size_t batch_update_entry_bytes();
tk_status batch_describe_raster(const tk_problem& p, void* dst);
tk_status batch_describe_update(const tk_problem& p, void* dst);
tk_status batch_launch_raster(const tk_problem* problems, int32_t n, const void* d_entries, hipStream_t s);
tk_status batch_launch_persistent(const tk_problem* problems, int32_t n, const void* d_entries, int32_t* d_counters,
                                  hipStream_t s);
tk_status batch_launch_tell(const tk_problem* problems, int32_t n, const void* d_entries, hipStream_t s);

tk_status validate_camera(const tk_camera* cam);
// Validates n_arms chains and fills a->ch, a->n_arms (and a->cam when cam is given).
tk_status make_fk_args(const tk_chain* chains, int32_t n_arms, const tk_camera* cam, FkArgs* a);
// Validates the loss-composition arguments and fills *la.
tk_status make_loss_args(int32_t batch, int32_t kind, double lambda_app, const float* d_kp, const float* d_kp_ref,
                         int32_t n_arms, double lambda_kp, double tau, LossArgs* la);
tk_status validate_meshes(const tk_mesh* meshes, int32_t n_meshes, MeshSet* out);

}  // namespace tk
