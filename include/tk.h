/*
 * tk.h -- C ABI of the MI355X (gfx950) batched silhouette-fitness library.
 *
 * The library evaluates, for lambda candidate states of a surgical instrument
 * (6-DoF look-at pose + 3 joint angles per arm), the silhouette-matching
 * objective of a CMA-ES tracker and runs the CMA-ES sample/update steps around
 * it (arXiv 2603.11404, Sec. III-A: problem statement Eq. (objective), CMA-ES
 * Eq. (cmaes_update), render loss Eq. (render_loss), renderer
 * S = R(K(Pi(T_r^c T_m^r(q) v_m))), state parameterisation; Sec. III-B
 * bi-manual block-diagonal covariance; Sec. IV mask error 1 - IoU).
 *
 * Conventions (all entry points):
 *   - Pointers named d_* are DEVICE pointers, caller-allocated and caller-
 *     freed.  Struct arguments (tk_camera, tk_mesh, tk_chain, ...) are HOST
 *     structs read during the call; the device pointers inside tk_mesh must
 *     stay valid until the queued work has run.
 *   - Work is queued on the given HIP stream (0 = legacy default stream);
 *     nothing synchronises the stream and no entry point allocates device
 *     memory.
 *   - Arguments are validated before anything is queued; on error nothing is
 *     queued, the status is returned and tk_last_error() (thread-local) holds a
 *     readable description.  A failed kernel launch returns TK_ERR_DEVICE.
 *   - Determinism: the same inputs (and, for CMA-ES, the same seed and
 *     generation) give bit-identical outputs.
 *   - Mask layout: a binary H x W image is stored as ceil(H/8) x ceil(W/8)
 *     uint64 words, row-major; pixel (x, y) is bit (y%8)*8 + (x%8) of word
 *     [y/8][x/8]; bits of pixels outside the image are zero.
 *   - Snapped vertices: Q8 fixed point, (X, Y) = rint(256 * clamp(u, +-32768))
 *     with ties to even; pixel (x, y) has its centre at (256x+128, 256y+128).
 *     A vertex that fails the near plane (or is not a number) is stored with
 *     X = INT32_MIN.
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* tk_stream; /* same type as hipStream_t */

/* Flag bit of the loss kind: the two-tip keypoint term of Eq. kpts_loss. */
#define TK_KP_TWO_TIPS 16

typedef enum {
    TK_OK = 0,
    TK_ERR_INVALID_ARGUMENT = 1,
    TK_ERR_UNSUPPORTED = 2,
    TK_ERR_WORKSPACE_TOO_SMALL = 3,
    TK_ERR_DEVICE = 4
} tk_status;

/* Static description of a status code. */
const char* tk_status_string(tk_status s);
/* Detail of the last error raised on the calling thread ("" if none). */
const char* tk_last_error(void);
/* Library version, e.g. 100 for 1.0.0. */
int32_t tk_version(void);

/* Pinhole camera K (Sec. III-A.2): u = fx*X/Z + cx, v = fy*Y/Z + cy, image y
 * pointing down; vertices with Z < z_near are culled with their triangles.
 * 1 <= width, height <= 4096. */
typedef struct { float fx, fy, cx, cy; int32_t width, height; float z_near; } tk_camera;

/* Instrument mesh v_m (Sec. III-A.2), device pointers:
 *   vertices [n_vertices][3] float32, metres, in the frame of their link;
 *   triangles [n_triangles][3] int32 vertex indices (either winding);
 *   vertex_link [n_vertices] uint8 in 0..3 (shaft, wrist, jaw+, jaw-).
 * 0 <= n_triangles <= 16M, 1 <= n_vertices <= 16M.
 * closed: 1 asserts that the triangles form a closed, consistently oriented
 * surface -- every directed edge a->b occurs as often as b->a, which
 * tk_mesh_closed checks on the host -- else 0.  For such a mesh the raster
 * entry points that snap through a workspace draw only the triangles of
 * positive signed area in the snapped image plane whenever no vertex of the
 * mesh fails the near plane: those cover exactly the pixel centres that all
 * triangles cover (the signed count of covering triangles at a centre,
 * taken at the infinitesimally shifted point that the top-left rule amounts
 * to, is the winding number of an empty boundary: zero), so the silhouette
 * is identical.  A wrong 1 gives wrong silhouettes. */
typedef struct {
    int32_t n_vertices, n_triangles;
    const float* vertices;
    const int32_t* triangles;
    const uint8_t* vertex_link;
    int32_t closed;
    int32_t reserved;   /* 0 */
} tk_mesh;

/* Kinematic chain of one instrument (Sec. III-A.3 and Fig. 2: end-effector
 * frame at the wrist pitch axis, z distal):
 *   shaft  T_0 = I;  wrist T_1 = Rx(q1);
 *   jaw+   T_2 = Rx(q1) Tr(0,0,d_pitch_yaw) Ry(q2 + q3/2);
 *   jaw-   T_3 = Rx(q1) Tr(0,0,d_pitch_yaw) Ry(q2 - q3/2).
 * q_lb/q_ub are the joint limits of the cosine map; keypoints[j] = (x, y, z in
 * metres in the frame of link id keypoints[j][3]). */
typedef struct {
    double d_pitch_yaw;
    double q_lb[3], q_ub[3];
    double keypoints[4][4];
} tk_chain;

/* ------------------------------------------------------------------ CMA-ES */

/* Multipliers on the default learning rates (paper Sec. IV raises c_m and
 * c_mu above their defaults without giving values; 1.0 = Hansen defaults) and
 * the number of diagonal covariance blocks (1, or 2 for the bi-manual
 * block-diagonal Sigma of Sec. III-B). */
typedef struct {
    double c_m_scale, c_mu_scale, c1_scale;
    int32_t n_blocks;
} tk_cmaes_params;

/* Byte offsets of the fields of the CMA-ES state blob (see tk_cmaes_layout).
 * Scalars are FP64 unless noted; matrices are row-major FP64. */
typedef struct {
    int64_t total_bytes;
    int64_t gen;        /* int64 generation counter g */
    int64_t seed;       /* uint64 Philox key */
    int64_t flags;      /* int32 bit 0: an eigenvalue or a Cholesky pivot was floored, bit 1: sigma or an
                         * eigenvalue not finite, bit 2: an internal wait of the update kernel
                         * exceeded its bound (the results of that update are not valid) */
    int64_t sigma, c_sigma, d_sigma, c_c, c1, c_mu, c_m, mu_eff, chi_n, h_sigma;
    int64_t weights;    /* [lambda] (first mu used) */
    int64_t mean, p_sigma, p_c, offset, scale, D;   /* [n] */
    int64_t C, B;       /* [n][n]; C the covariance the next candidates are drawn with; B, D the
                         * eigendecomposition (B columns eigenvectors, D square roots of the
                         * eigenvalues) of the covariance the last update whitened with, i.e. the
                         * one before it (identity after initialisation) */
    int64_t Z, Y;       /* [lambda][n] last draws z and y = L z */
    int64_t order;      /* int32 [lambda] ranking of the last update */
    int64_t z_gen;      /* int64 generation g whose draws Z holds for every candidate (-1: none,
                         * or older than the draws in Z).  An update with n <= 9 draws the
                         * next generation's z beside its eigendecomposition and the
                         * ask-eval form then reads them; otherwise the ask-eval prologue
                         * draws them itself (and does not tag them), as do the sampler
                         * and the tell-ask form (which tag them) */
    int64_t L;          /* [n][n] lower Cholesky factor of C per diagonal block (L L^T = C; zero
                         * above the diagonal and off the blocks), the sampling square root */
} tk_cmaes_layout;

/* Size in bytes of a state blob for dimension n (1..18) and population
 * lambda (2..1024); 0 on invalid sizes. */
size_t tk_cmaes_state_bytes(int32_t n, int32_t lambda);
tk_status tk_cmaes_layout_get(int32_t n, int32_t lambda, tk_cmaes_layout* out);

/* Initialise a state blob (Sec. III-A.1; Sec. IV: Sigma^(0) = I in the
 * normalised space): m = mean0 (normalised space, host [n]), sigma = sigma0,
 * C = L = B = I, D = 1, p_sigma = p_c = 0, g = 0.  Physical candidates are
 * theta = offset + scale * x (host [n] each).  p may be NULL for defaults.
 * n must be divisible by p->n_blocks. */
tk_status tk_cmaes_init(void* d_state, int32_t n, int32_t lambda, const double* mean0, double sigma0,
                        const double* offset, const double* scale, const tk_cmaes_params* p,
                        uint64_t seed, tk_stream s);

/* Initialise a state blob for the next frame at an estimate that is already
 * in device memory, so a frame loop needs no host round trip (Sec. III-A: each
 * frame starts from the previous frame's estimate; Sec. III-A.3: cosine joint
 * map).  d_est: device FP64 [n], n = 9 n_arms, in the temporal filter's
 * coordinates (pose, then joint angles q per arm), e.g. the theta or
 * theta_next output of tk_kf_step.  The offset of each coordinate is
 * d_est[i] for the pose and the inverse cosine map of the clamped joint angle
 * (limits from chains, host [n_arms]) for the joints; where readings (host
 * [n_arms][3] unconstrained joint coordinates, may be NULL) are given they
 * replace the joint offsets.  Otherwise as tk_cmaes_init with mean0 = 0:
 * sigma = sigma0, scale (host [n]), C = L = B = I, D = 1, paths 0, g = 0, seed,
 * p (may be NULL).  d_est is read by the launched kernel, in stream order.
 * Errors: TK_ERR_INVALID_ARGUMENT on sizes, NULL pointers, non-finite scale or
 * readings, joint limits with lb >= ub; nothing is launched then. */
tk_status tk_cmaes_init_at(void* d_state, int32_t n, int32_t lambda, const double* d_est, const tk_chain* chains,
                           int32_t n_arms, const double* readings, double sigma0, const double* scale,
                           const tk_cmaes_params* p, uint64_t seed, tk_stream s);

/* Replace the mean (normalised space, host [n]) without touching sigma, C or
 * the paths (warm start from the previous frame, Sec. III-A). */
tk_status tk_cmaes_set_mean(void* d_state, int32_t n, int32_t lambda, const double* mean, tk_stream s);

/* Sample lambda candidates from N(m, sigma^2 C) (Sec. III-A.1, Eq.
 * expected_fitness): z from Philox4x32-10 (key = seed, counter = (j, k, g, 0))
 * with Box-Muller, y = L z (L L^T = C, so y ~ N(0, C)), x = m + sigma y.  Writes d_X[lambda][n] FP32
 * physical candidates theta = offset + scale * x and keeps z, y in the state. */
tk_status tk_cmaes_sample(void* d_state, int32_t n, int32_t lambda, float* d_X, tk_stream s);

/* One CMA-ES update from the losses of the last sample (Sec. III-A.1, Eq.
 * cmaes_update, completed by Hansen's tutorial): rank by (loss, index) with
 * NaN as +inf, weighted recombination of the mu = lambda/2 best, cumulative
 * step-size adaptation with C^(-1/2) from the Jacobi eigendecomposition of the
 * covariance the candidates were drawn with, rank-one + rank-mu covariance
 * update, symmetrisation, optional block-diagonal masking (Sec. III-B), and
 * the Cholesky factor L of the new covariance for the next draws (pivots
 * floored at 1e-20 max_i C_ii).  d_loss: device FP64 [lambda]. */
tk_status tk_cmaes_update(void* d_state, int32_t n, int32_t lambda, const double* d_loss, tk_stream s);

/* Loss composition and update in one launch ("tell"), identical to
 *   tk_compose_loss(d_counts, lambda, d_target_count, kind, lambda_app, d_kp,
 *                   d_kp_ref, n_arms, lambda_kp, tau, d_loss)
 *   tk_cmaes_update(d_state, n, lambda, d_loss)
 * (Eq. (3)-(4), (5)-(8)).  d_loss (FP64 [lambda]) is an optional output. */
tk_status tk_cmaes_tell(void* d_state, int32_t n, int32_t lambda, const int32_t* d_counts,
                        const int32_t* d_target_count, int32_t kind, double lambda_app, const float* d_kp,
                        const float* d_kp_ref, int32_t n_arms, double lambda_kp, double tau, double* d_loss,
                        tk_stream s);

/* Fused generation step ("tell" the losses of the evaluated candidates, "ask"
 * for the next ones) in one launch, with results identical to the sequence
 *   tk_compose_loss(d_counts, lambda, d_target_count, kind, lambda_app, d_kp,
 *                   d_kp_ref, n_arms, lambda_kp, tau, d_loss)
 *   tk_cmaes_update(d_state, n, lambda, d_loss)
 *   tk_cmaes_sample(d_state, n, lambda, d_X)
 *   tk_fk_transform(d_X, lambda, n_arms, chains, d_link_xf, d_kp_next, cam)
 * (Eq. (3)-(4) and (5)-(8), Sec. III-A.3).  n must be 9 * n_arms.  d_loss
 * (FP64 [lambda]) and d_kp_next are optional outputs; d_kp / d_kp_ref are the
 * evaluated candidates' keypoints and the reference (both or neither); d_kp
 * and d_kp_next may be the same buffer (read before written).  cam is
 * required.  All pointers are device pointers except chains and cam. */
tk_status tk_cmaes_tell_ask(void* d_state, int32_t n, int32_t lambda, const int32_t* d_counts,
                            const int32_t* d_target_count, int32_t kind, double lambda_app, const float* d_kp,
                            const float* d_kp_ref, double lambda_kp, double tau, double* d_loss,
                            const tk_chain* chains, int32_t n_arms, const tk_camera* cam, float* d_X,
                            float* d_link_xf, float* d_kp_next, tk_stream s);

/* ------------------------------------------------------- fitness evaluation */

/* Forward kinematics (Sec. III-A.3 and the renderer input T_r^c T_m^r(q)):
 * d_X[batch][9*n_arms] FP32 candidates (alpha, beta, gamma, x, y, z, qhat1..3
 * per arm) -> d_link_xf[batch][n_arms][4][12] FP32 row-major 3x4 transforms
 * M_l = T_r^c(alpha,beta,gamma,x,y,z) T_l(q), q from the cosine map; computed
 * in FP32.  d_kp (nullable) [batch][n_arms][4][2] FP32 projected
 * chain keypoints (NaN when behind z_near).  chains: host [n_arms]. */
tk_status tk_fk_transform(const float* d_X, int32_t batch, int32_t n_arms, const tk_chain* chains,
                          float* d_link_xf, float* d_kp, const tk_camera* cam, tk_stream s);

/* Transform, project and snap every vertex (FP32 transform, Q8 snap):
 * d_snapped[batch][sum of n_vertices][2] int32 (arms concatenated). */
tk_status tk_snap_vertices(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                           const tk_camera* cam, int32_t* d_snapped, tk_stream s);

/* Workspace bytes that let the raster entry points snap each vertex once per
 * candidate (batch * total vertices * 8); 0 on invalid arguments. */
size_t tk_raster_workspace_bytes(int32_t batch, const tk_mesh* meshes, int32_t n_meshes);

/* Claim order of a mesh's triangles for the raster entry points (the silhouette
 * S of Sec. III-A.2 is an OR over triangles, so any order renders the same
 * mask).  HOST pointers, no device call: vertices [n_vertices][3] and
 * triangles [n_triangles][3] as in tk_mesh; triangles_out [n_triangles][3]
 * (caller-owned, must not overlap triangles) receives the same triangles in
 * blocks of 64 cut from the end of the list, the full blocks by decreasing
 * summed model-space area, then the short block of the first n_triangles mod
 * 64 triangles.  The raster kernels claim 64-triangle chunks in list order, so
 * a mesh stored this way is rasterised costly chunks first, and the waves end
 * close together.  Errors: TK_ERR_INVALID_ARGUMENT on sizes, NULL pointers,
 * overlap or a vertex index outside [0, n_vertices); triangles_out is then
 * not written. */
tk_status tk_mesh_chunk_order(const float* vertices, int32_t n_vertices, const int32_t* triangles,
                              int32_t n_triangles, int32_t* triangles_out);

/* Whether a triangle list (HOST [n_triangles][3], indices in [0, n_vertices))
 * is a closed, consistently oriented surface: *closed = 1 when every
 * directed edge a->b occurs exactly as often as b->a (edges of a repeated
 * vertex are ignored), else 0 -- the value tk_mesh.closed asserts.
 * Errors: TK_ERR_INVALID_ARGUMENT on sizes, NULL pointers or indices out of
 * range; *closed is then not written. */
tk_status tk_mesh_closed(const int32_t* triangles, int32_t n_triangles, int32_t n_vertices, int32_t* closed);

/* Plane order of a mesh's triangles (HOST pointers, no device call; same
 * silhouette in any order): triangles_out [n_triangles][3] receives the
 * triangles sorted by their supporting plane in model space -- the link of
 * their first vertex, the direction of the unit normal (2-degree polar bands,
 * then 0.01-degree azimuth bins), then the plane's offset (0.1 micrometre
 * bins); ties keep list order; degenerate triangles last in their link.
 * Coplanar triangles of one link project with the same orientation in every
 * pose, so 64-triangle chunks of this order are mostly wholly back-facing or
 * wholly front-facing, and the one-sided raster path (tk_mesh.closed) skips
 * back-facing chunks as a whole.  Apply before tk_mesh_chunk_order, which
 * moves whole 64-triangle blocks.  Errors as for tk_mesh_chunk_order. */
tk_status tk_mesh_plane_order(const float* vertices, const uint8_t* vertex_link, int32_t n_vertices,
                              const int32_t* triangles, int32_t n_triangles, int32_t* triangles_out);

/* Binary silhouette S (Sec. III-A.2: S in {0,1}^{H x W}) of every candidate:
 * OR over the n_meshes arms (one mesh per arm, link transforms from
 * d_link_xf[batch][n_meshes][4][12]) of the exact integer coverage with the
 * top-left fill rule, both windings drawn, no depth test.
 * d_masks [batch][ceil(H/8)][ceil(W/8)] uint64.  The image mask lives in LDS:
 * ceil(H/8)*ceil(W/8)*8 bytes must stay below about 136 KB (1280x720 fits;
 * larger images return TK_ERR_UNSUPPORTED).  Triangle indices must lie in
 * [0, n_vertices).  d_ws (nullable, device, tk_raster_workspace_bytes) holds
 * the snapped vertices between the two phases of the kernel; with NULL each
 * triangle transforms its own vertices (same result, more arithmetic);
 * a smaller workspace returns TK_ERR_WORKSPACE_TOO_SMALL. */
tk_status tk_raster_silhouette(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                               const tk_camera* cam, uint64_t* d_masks, void* d_ws, size_t ws_bytes, tk_stream s);

/* Same coverage from given snapped vertices d_snapped[batch][sum V][2]. */
tk_status tk_raster_from_snapped(const int32_t* d_snapped, int32_t batch, const tk_mesh* meshes,
                                 int32_t n_meshes, const tk_camera* cam, uint64_t* d_masks, tk_stream s);

/* Counts of the render loss (Eq. render_loss) against the observed mask
 * M_ref: d_counts[batch][2] int32 = {|S|, |S and M|}.  d_target: one mask. */
tk_status tk_mask_loss(const uint64_t* d_masks, int32_t batch, const uint64_t* d_target, const tk_camera* cam,
                       int32_t* d_counts, tk_stream s);

/* d_count[batch] int32 = |S| for each mask (e.g. the target count |M|). */
tk_status tk_mask_popcount(const uint64_t* d_masks, int32_t batch, const tk_camera* cam, int32_t* d_count,
                           tk_stream s);

/* Fused raster + counts: d_link_xf -> d_counts[batch][2] without writing
 * masks (same coverage as tk_raster_silhouette followed by tk_mask_loss);
 * workspace as for tk_raster_silhouette. */
tk_status tk_eval_fused(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                        const tk_camera* cam, const uint64_t* d_target, int32_t* d_counts, void* d_ws,
                        size_t ws_bytes, tk_stream s);

/* Sampling and evaluation of a whole generation in one launch ("ask" and
 * evaluate), one workgroup per candidate, identical to
 *   tk_cmaes_sample(d_state, n, lambda, d_X)
 *   tk_fk_transform(d_X, lambda, n_arms, chains, d_link_xf, d_kp, cam)
 *   tk_eval_fused(d_link_xf, lambda, meshes, n_arms, cam, d_target, d_counts,
 *                 d_ws, ws_bytes)
 * (Eq. (3)-(4) sampling, Sec. III-A.3, Eq. (7), Eq. (6) counts).  n must be
 * 9 * n_arms, one mesh per arm; d_kp (nullable) receives the keypoints;
 * workspace as for tk_eval_fused. */
tk_status tk_cmaes_ask_eval(void* d_state, int32_t n, int32_t lambda, const tk_chain* chains, int32_t n_arms,
                            const tk_mesh* meshes, const tk_camera* cam, const uint64_t* d_target, float* d_X,
                            float* d_link_xf, float* d_kp, int32_t* d_counts, void* d_ws, size_t ws_bytes,
                            tk_stream s);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * launch and results as tk_cmaes_ask_eval with a workspace, but the
 * snapped-vertex workspace is a static array inside the library, one per
 * device, of TK_NOALLOC_SCRATCH_BYTES (allocated when the library's code
 * object is loaded on a device and held until the process ends; its address
 * is looked up on the first call on each device).  The call allocates
 * nothing.  Requires lambda * (sum of the meshes' n_vertices) * 8 <=
 * TK_NOALLOC_SCRATCH_BYTES (e.g. 256 candidates of a 10k-vertex mesh), else
 * TK_ERR_UNSUPPORTED and nothing is launched.  Every call on a device uses
 * that device's one array: calls whose launches overlap on one device (other
 * streams, other threads) race and give undefined counts; calls ordered on a
 * stream are fine.  The kernel writes every entry it reads before reading it,
 * so nothing needs clearing between calls.  Other arguments and errors as for
 * tk_cmaes_ask_eval. */
#define TK_NOALLOC_SCRATCH_BYTES (32 * 1024 * 1024)
tk_status tk_cmaes_ask_eval_noalloc(void* d_state, int32_t n, int32_t lambda, const tk_chain* chains,
                                    int32_t n_arms, const tk_mesh* meshes, const tk_camera* cam,
                                    const uint64_t* d_target, float* d_X, float* d_link_xf, float* d_kp,
                                    int32_t* d_counts, tk_stream s);

/* Workload statistics of a raster launch over the same inputs (for
 * measurement, not on the hot path): d_stats[4] uint64 = {triangles kept,
 * pixel centres inside the kept triangles' clamped boxes, (triangle, 8x8
 * block) pairs visited, triangles needing 64-bit edge functions}.  The
 * counters are cleared on the stream first. */
tk_status tk_raster_stats(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                          const tk_camera* cam, uint64_t* d_stats, tk_stream s);

/* Bandwidth microbenchmarks for the roofline denominators (measurement only,
 * not on the fitness path).  tk_bench_copy: a streaming copy of bytes (a
 * multiple of 16; 16-byte aligned device pointers) from d_src to d_dst --
 * 2 * bytes of HBM traffic.  tk_bench_lds: `workgroups` workgroups of 256
 * threads, each with 64 KB of LDS, run `iters` iterations of 4 conflict-free
 * 128-bit LDS reads and 4 writes per thread (iters * 256 * 128 bytes per
 * workgroup) and XOR their data into d_out[workgroup] (device uint32
 * [workgroups], caller-cleared).  Errors: TK_ERR_INVALID_ARGUMENT. */
tk_status tk_bench_copy(const void* d_src, void* d_dst, size_t bytes, tk_stream s);
tk_status tk_bench_lds(int32_t workgroups, int32_t iters, uint32_t* d_out, tk_stream s);

/* Loss composition in FP64 (Eq. objective and render_loss; Sec. IV):
 *   kind 0: 1 - IoU = 1 - i/(a + m - i)  (0 when the union is empty);
 *   kind 1: (a + m - 2i) + lambda_app*|a - m|  (sum of squared mask errors
 *           plus the appearance term, exact on binary masks);
 * plus, when d_kp and d_kp_ref are given and lambda_kp != 0, lambda_kp times
 * the keypoint term of every arm (Eq. kpts_loss extended to the 4 chain
 * keypoints: (|p_j - r_j| - tau)_+ for the shaft and wrist keypoints, the
 * better of the two jaw-tip assignments, and the tip-midpoint term).
 * kind | TK_KP_TWO_TIPS takes Eq. kpts_loss as printed instead: the two jaw
 * tips (keypoints 2, 3) under the better assignment plus their midpoint, and
 * no keypoint term for an arm unless its two reference tips are finite and
 * distinct (the paper evaluates the term only for exactly two detections).
 * The kind argument of tk_cmaes_tell, tk_cmaes_tell_ask and tk_problem takes
 * the same values.
 * d_counts [batch][2] from tk_mask_loss, d_target_count: device int32 |M|,
 * d_kp [batch][n_arms][4][2], d_kp_ref [n_arms][4][2], d_loss [batch] FP64. */
tk_status tk_compose_loss(const int32_t* d_counts, int32_t batch, const int32_t* d_target_count, int32_t kind,
                          double lambda_app, const float* d_kp, const float* d_kp_ref, int32_t n_arms,
                          double lambda_kp, double tau, double* d_loss, tk_stream s);

/* ------------------------------------------------------- differentiable form */

/* Soft silhouette (a differentiable stand-in for the renderer of Sec.
 * III-A.2; loss = the squared-error term of Eq. (6) summed over the pixels):
 * for the pixel centre p and face j of any arm (FP32 projected corners, no
 * snapping; faces with a corner in front of z_near or of zero area left out),
 * d_j(p) is the signed distance to the face boundary (positive inside),
 * prob_j = (sig(d_j / sigma) - s0) / (1 - s0) for d_j >= -10 sigma and 0
 * below (s0 = sig(-10), so prob reaches 0 at the cutoff), S(p) = 1 -
 * prod_j (1 - prob_j) and L = sum_p (S(p) - M(p))^2 per candidate.
 * Deterministic: the per-pixel sums are taken in 64-bit fixed point and every
 * other reduction in a fixed order.  Images up to 16384 8x8 tiles (1024x1024;
 * larger return TK_ERR_UNSUPPORTED). */

/* Workspace bytes of tk_soft_forward / tk_soft_backward for batch candidates
 * (0 on invalid arguments).  It holds the projected corners, face records,
 * tile lists (up to 32 tiles per face; larger faces on a per-candidate list),
 * the per-pixel factor 2 (S - M)(1 - S) / sigma and partial sums. */
size_t tk_soft_workspace_bytes(int32_t batch, const tk_mesh* meshes, int32_t n_meshes, const tk_camera* cam);

/* Forward pass: d_link_xf [batch][n_meshes][4][12] (tk_fk_transform), one
 * observed word mask d_target, sigma in pixels (0 < sigma <= 64).  Writes
 * d_loss [batch] FP64 and, when d_S is not NULL, S [batch][H][W] FP32; keeps in
 * d_ws (256-byte aligned, tk_soft_workspace_bytes) what the backward pass
 * reads. */
tk_status tk_soft_forward(const float* d_link_xf, int32_t batch, const tk_mesh* meshes, int32_t n_meshes,
                          const tk_camera* cam, float sigma, const uint64_t* d_target, float* d_S, double* d_loss,
                          void* d_ws, size_t ws_bytes, tk_stream s);

/* Backward pass of the last tk_soft_forward on the same workspace, meshes,
 * camera and sigma: d_grad_X [batch][9 n_arms] FP32 = dL/dtheta of the
 * candidates d_X [batch][9 n_arms] (the theta the link transforms came from),
 * through the pinhole projection, the link transforms and the forward
 * kinematics with the cosine joint map (Sec. III-A.3), scaled per candidate
 * by d_grad_loss [batch] FP64 when not NULL.  chains: host [n_arms]. */
tk_status tk_soft_backward(const float* d_X, int32_t batch, const tk_chain* chains, const tk_mesh* meshes,
                           int32_t n_arms, const tk_camera* cam, float sigma, const double* d_grad_loss,
                           float* d_grad_X, void* d_ws, size_t ws_bytes, tk_stream s);

/* The CMA-ES mean as an FP32 candidate: d_X[i] = offset_i + scale_i m_i. */
tk_status tk_cmaes_mean_candidate(const void* d_state, int32_t n, int32_t lambda, float* d_X, tk_stream s);

/* Zero an Adam state of dimension n (device, 8 (2n + 1) bytes: m, v, t). */
tk_status tk_adam_reset(void* d_adam, int32_t n, tk_stream s);

/* One Adam step (Kingma and Ba: m, v moments, bias correction) on the CMA-ES
 * mean in the normalised space x (theta = offset + scale x), from d_grad_theta
 * [n] FP32 = dL/dtheta at the mean (gradient in x = gradient in theta x
 * scale).  Only the mean of the state changes. */
tk_status tk_cmaes_adam(void* d_state, int32_t n, int32_t lambda, const float* d_grad_theta, void* d_adam,
                        double lr, double beta1, double beta2, double eps, tk_stream s);

/* One refinement step in one launch: when d_grad_theta is not NULL, the Adam
 * step of tk_cmaes_adam (same arithmetic, d_adam required); then the mean as
 * an FP32 candidate (tk_cmaes_mean_candidate) into d_X [9 n_arms] and, when
 * d_link_xf is not NULL, its link transforms [n_arms][4][12]
 * (tk_fk_transform of that candidate; chains: host [n_arms]).  n must be
 * 9 n_arms.  Bit-identical to the separate calls in that order. */
tk_status tk_cmaes_adam_transform(void* d_state, int32_t n, int32_t lambda, const float* d_grad_theta,
                                  void* d_adam, double lr, double beta1, double beta2, double eps, int32_t n_arms,
                                  const tk_chain* chains, float* d_X, float* d_link_xf, tk_stream s);

/* ------------------------------------------------------- temporal filter */

/* Constant-velocity Kalman filter of the per-frame estimates (Sec. III-A.4,
 * Eq. kf_motion and the observation model that follows it): state
 * s_t = [theta_t; theta_dot_t] (2n), s_t = [[I, dt I], [0, I]] s_{t-1} + w_t,
 * w_t ~ N(0, Q), observation z_t = [I 0] s_t + v_t, v_t ~ N(0, R), then the
 * filtered theta is clamped to [lo, hi] per coordinate.  Supported noise:
 * Q = [[diag(q_pos), diag(q_cross)], [diag(q_cross), diag(q_vel)]] and
 * R = diag(r), with P0 = diag(p0_pos, p0_vel); under these the filter is n
 * independent 2-state filters, which the device evaluates in FP64, one lane
 * per coordinate.  A non-finite z_i is a missing measurement: coordinate i is
 * predicted only.  All arrays hold n used entries (n <= 18). */
#define TK_KF_MAX_N 18
typedef struct {
    double dt;                                   /* frame interval, > 0 */
    double p0_pos[TK_KF_MAX_N], p0_vel[TK_KF_MAX_N];   /* >= 0 */
    double q_pos[TK_KF_MAX_N], q_cross[TK_KF_MAX_N], q_vel[TK_KF_MAX_N];  /* PSD 2x2 blocks */
    double r[TK_KF_MAX_N];                       /* > 0 */
    double lo[TK_KF_MAX_N], hi[TK_KF_MAX_N];     /* clamp limits; +-INFINITY for none */
} tk_kf_params;

/* Bytes of the device filter state for n coordinates (0 unless 1 <= n <= 18). */
size_t tk_kf_state_bytes(int32_t n);

/* (Re)start the filter at theta = x0 (host [n], inside [lo, hi]) with zero
 * velocity and covariance P0; params: host.  d_kf: device, tk_kf_state_bytes.
 * Errors: TK_ERR_INVALID_ARGUMENT on sizes, NULL pointers, non-finite values,
 * a non-PSD noise block, r <= 0 or lo > hi; nothing is launched then. */
tk_status tk_kf_init(void* d_kf, int32_t n, const double* x0, const tk_kf_params* p, tk_stream s);

/* One frame: predict, update with d_z (device FP64 [n]), clamp.  Writes the
 * filtered theta_t to d_theta and the clamped constant-velocity prediction
 * theta_t + dt * theta_dot_t for the next frame to d_theta_next (device FP64
 * [n] each, both nullable).  n must be the value given to tk_kf_init. */
tk_status tk_kf_step(void* d_kf, int32_t n, const double* d_z, double* d_theta, double* d_theta_next,
                     tk_stream s);

/* The CMA-ES estimate of a frame as the filter's measurement: d_z[i] =
 * offset_i + scale_i * m_i (device FP64 [n]), with the three joint coordinates
 * of every arm taken through the cosine map of Sec. III-A.3 into joint angles
 * in [q_lb, q_ub] (FP64).  n must be 9 * n_arms; chains: host [n_arms]. */
tk_status tk_cmaes_estimate(const void* d_state, int32_t n, int32_t lambda, const tk_chain* chains,
                            int32_t n_arms, double* d_z, tk_stream s);

/* ------------------------------------------------------- batched problems */

/* One independent tracking problem of a batched launch (host struct holding
 * device pointers; NEXT batching form of the tracker, Sec. III-A.1 run for
 * many problems at once): its CMA-ES state (n = 9 * n_arms, lambda), one mesh
 * and one chain per arm, camera, observed mask and |M|, and the buffers of its
 * candidates exactly as for tk_cmaes_ask_eval (d_X, d_link_xf, d_kp nullable,
 * d_counts, workspace d_ws / ws_bytes required) and tk_cmaes_tell (kind,
 * lambda_app, d_kp_ref nullable, lambda_kp, tau, d_loss nullable).  threads:
 * raster workgroup size, 0 = the widest whose LDS fits, else 256, 512, 1024
 * (a tuning choice; results do not depend on it). */
typedef struct {
    void* d_state;
    int32_t n, lambda, n_arms;
    tk_mesh meshes[2];
    tk_chain chains[2];
    tk_camera cam;
    const uint64_t* d_target;
    const int32_t* d_target_count;
    float* d_X;
    float* d_link_xf;
    float* d_kp;
    int32_t* d_counts;
    void* d_ws;
    size_t ws_bytes;
    int32_t kind;
    double lambda_app;
    const float* d_kp_ref;
    double lambda_kp;
    double tau;
    double* d_loss;
    int32_t threads;
} tk_problem;

/* Bytes of the device table of n_problems (0 if n_problems is outside
 * 1..65536): problem descriptors and the control words of the persistent
 * launch. */
size_t tk_batch_table_bytes(int32_t n_problems);

/* Validates the problems and writes their device descriptors into the HOST
 * buffer h_table (256-byte aligned, tk_batch_table_bytes); the caller copies
 * it to a 256-byte aligned device buffer, which the batched calls read.  The
 * table stays valid as long as the problems' device buffers do. */
tk_status tk_batch_describe(const tk_problem* problems, int32_t n_problems, void* h_table, size_t table_bytes);

/* tk_cmaes_ask_eval for every problem, with identical results; problems of
 * one workgroup size share a launch (at most 128 problems per launch).
 * problems: the host array given to tk_batch_describe; d_table: its device
 * copy. */
tk_status tk_batch_ask_eval(const tk_problem* problems, int32_t n_problems, const void* d_table, tk_stream s);

/* tk_cmaes_ask_eval for every problem, with identical results, in one
 * persistent launch per 128 problems (NEXT batching form: candidates of all
 * problems, of any image size and mesh, in one launch): a resident grid of
 * 1024-thread workgroups, one per compute unit, claims (problem, candidate)
 * items from a counter in d_table, the problems ordered costliest per
 * candidate first (image pixels x sqrt(triangles)); each item lays out its
 * LDS for its image (mask, then per-wave task rings: 128 narrow slots for 16
 * rasterising waves where they fit, else 64 slots for as many waves as fit).
 * The problems' threads field is not used.  d_table: the device copy of the
 * tk_batch_describe table, NOT const: its control words (zero in the
 * described table) count the claims and are reset to zero by the launch's
 * last workgroup, so launches on one table must not overlap.  Errors as for
 * tk_batch_ask_eval; TK_ERR_UNSUPPORTED when an image leaves no LDS for one
 * wave's queues (above about 1700 x 1000 pixels). */
tk_status tk_batch_ask_eval_persistent(const tk_problem* problems, int32_t n_problems, void* d_table, tk_stream s);

/* tk_cmaes_tell for every problem, with identical results: one workgroup per
 * problem, one launch per 128 problems (per covariance size class). */
tk_status tk_batch_tell(const tk_problem* problems, int32_t n_problems, const void* d_table, tk_stream s);

#ifdef __cplusplus
}
#endif
#endif
