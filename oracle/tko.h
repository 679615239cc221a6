/*
 * tko.h -- CPU oracle for the batched silhouette-fitness path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * bench's CPU-baseline leg may load this library.  It shares no code with the
 * GPU library: plain C99, FP64 transforms, int64 rasterisation.
 *
 * Paper sections followed (arXiv 2603.11404):
 *   Sec. III-A.3 (state parameterisation: look-at rotation, cosine joint map),
 *   Sec. III-A.2 (renderer S = R(K(Pi(T_r^c T_m^r(q) v_m))), render loss),
 *   Sec. IV (mask error 1 - IoU, keypoint reprojection error),
 *   and a soft (differentiable) silhouette with its gradient (tko_soft.c).
 */
#ifndef TKO_H
#define TKO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double fx, fy, cx, cy; int32_t width, height; double z_near; } tko_camera;
/* keypoints[j] = {x, y, z (link frame, metres), link id} */
typedef struct { double d_pitch_yaw; double q_lb[3], q_ub[3]; double keypoints[4][4]; } tko_chain;

/* Cosine joint map (Sec. III-A.3): qhat -> q in [lb, ub] and its inverse. */
double tko_decode(double qhat, double lb, double ub);
double tko_encode(double q, double lb, double ub);

/* Look-at pose T_r^c as a 3x4 row-major [R | t]; R = Ry(gamma) Rx(alpha) Rz(beta). */
void tko_pose(double alpha, double beta, double gamma, double x, double y, double z, double T[12]);

/* Link transforms T_l (robot frame), l = shaft, wrist, jaw+, jaw-, from q. */
void tko_chain_links(const double q[3], const tko_chain* ch, double T[4][12]);

/* theta[9] = (alpha, beta, gamma, x, y, z, qhat1..3) -> M_l = T_r^c T_l, 3x4 each. */
void tko_fk(const double theta[9], const tko_chain* ch, double M[4][12]);

/* Transform, project and snap V vertices.  uv[V][2] (nullable) gets the
 * projected FP64 pixel coordinates, snapped[V][2] the Q8 fixed-point
 * coordinates rint(256*clamp(u)), flags[V] = 1 where the vertex is in front of
 * z_near fails (or is not a number). */
void tko_project_snap(const double M[4][12], const float* vertices, const uint8_t* vlink, int32_t V,
                      const tko_camera* cam, double* uv, int32_t* snapped, uint8_t* flags);

/* Project the chain keypoints through M (no snapping): kp[4][2]; NaN if behind z_near. */
void tko_keypoints(const double M[4][12], const tko_chain* ch, const tko_camera* cam, double kp[4][2]);

/* Rasterise one mesh from snapped vertices into a word mask (OR into mask,
 * layout [ceil(H/8)][ceil(W/8)] words, bit ly*8+lx).  counts (nullable, [H][W])
 * is incremented once per covering triangle.  Returns the number of triangles
 * that were not culled. */
int64_t tko_raster(const int32_t* snapped, const uint8_t* flags, int32_t V,
                   const int32_t* tris, int32_t T, int32_t W, int32_t H,
                   uint64_t* mask, int32_t* counts);

/* out = {|S|, |S and M|, |M|} over the valid pixels. */
void tko_counts(const uint64_t* S, const uint64_t* M, int32_t W, int32_t H, int64_t out[3]);

/* Loss from counts: kind 0 = 1 - IoU (IoU := 1 on an empty union),
 * kind 1 = render loss (xor count + lambda_app * |a - m|). */
double tko_mask_loss(int64_t a, int64_t i, int64_t m, int32_t kind, double lambda_app);

/* Keypoint term: two fixed keypoints (0, 1) plus the jaw tips (2, 3) matched
 * under the better of the two assignments, plus the tip-midpoint term, each
 * as (distance - tau)_+ in pixels. */
double tko_kp_loss(const double kp[4][2], const double ref[4][2], double tau);

/* Keypoint loss of Eq. (8) on the two tool tips (keypoints 2 and 3) only:
 * min over the two assignments of the sum of (distance - tau)_+ plus the
 * tip-midpoint term; 0 unless the two reference tips are finite and distinct. */
double tko_kp_loss_tips(const double kp[4][2], const double ref[4][2], double tau);

/* Whole candidate evaluation used for the CPU baseline:
 * for b in [0, batch): theta[b][n_arms*9] -> FK -> project/snap -> raster (OR of
 * the arms' meshes) -> counts[b][2] = {|S|, |S and M|}.  Runs the candidates
 * in parallel over n_threads OpenMP threads (<= 0: library default). */
typedef struct { int32_t n_vertices, n_triangles; const float* vertices; const int32_t* triangles;
                 const uint8_t* vertex_link; } tko_mesh;
void tko_eval_batch(const double* theta, int32_t batch, int32_t n_arms, const tko_chain* chains,
                    const tko_mesh* meshes, const tko_camera* cam, const uint64_t* target,
                    int64_t* counts, uint64_t* masks_out /* nullable [batch][words] */,
                    int32_t n_threads);
int32_t tko_max_threads(void);

/* Jacobian of the link transforms of tko_fk: dM[k][l] = d M_l / d theta_k
 * (theta as for tko_fk, joints through the cosine map), 3x4 each. */
void tko_fk_jacobian(const double theta[9], const tko_chain* ch, double dM[9][4][12]);

/* Soft silhouette of the arms at theta[n_arms * 9] (definition in
 * tko_soft.c): returns L = sum_p (S(p) - M(p))^2 over the image, with M the
 * word mask target (NULL: all zero).  S_out (nullable, [H][W]) gets S;
 * grad (nullable, [n_arms * 9]) gets dL/dtheta. */
#define TKO_SOFT_MAXP 18
double tko_soft(const double* theta, int32_t n_arms, const tko_chain* chains, const tko_mesh* meshes,
                const tko_camera* cam, double sigma, const uint64_t* target, double* S_out, double* grad);

/* The same S, loss and gradient evaluated face-major over each face's box
 * grown by 10 sigma (tko_soft_banded in tko_soft.c): S and L are the same
 * numbers as tko_soft's; the gradient agrees to rounding.  For large meshes. */
double tko_soft_banded(const double* theta, int32_t n_arms, const tko_chain* chains, const tko_mesh* meshes,
                       const tko_camera* cam, double sigma, const uint64_t* target, double* S_out, double* grad);

#ifdef __cplusplus
}
#endif
#endif
