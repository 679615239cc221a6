// Status strings, thread-local error detail and shared argument validation.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "tk_internal.h"

namespace tk {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

tk_status fail(tk_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

tk_status check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(TK_ERR_DEVICE, "%s: launch failed: %s", what, hipGetErrorString(e));
    return TK_OK;
}

tk_status validate_camera(const tk_camera* cam) {
    TK_REQUIRE(cam != nullptr, "camera is NULL");
    TK_REQUIRE(cam->width >= 1 && cam->width <= kMaxImage && cam->height >= 1 && cam->height <= kMaxImage,
               "image size %dx%d outside 1..%d", cam->width, cam->height, kMaxImage);
    TK_REQUIRE(cam->fx == cam->fx && cam->fy == cam->fy && cam->cx == cam->cx && cam->cy == cam->cy,
               "camera intrinsics are NaN");
    TK_REQUIRE(cam->z_near > 0.0f, "z_near must be > 0");
    return TK_OK;
}

tk_status make_fk_args(const tk_chain* chains, int32_t n_arms, const tk_camera* cam, FkArgs* a) {
    TK_REQUIRE(n_arms >= 1 && n_arms <= kMaxArms, "n_arms = %d outside 1..%d", n_arms, kMaxArms);
    TK_REQUIRE(chains != nullptr, "chains is NULL");
    std::memset(a, 0, sizeof *a);
    if (cam) {
        if (tk_status st = validate_camera(cam)) return st;
        a->cam = make_cam(*cam);
    }
    for (int i = 0; i < n_arms; i++) {
        const tk_chain& c = chains[i];
        TK_REQUIRE(std::isfinite(c.d_pitch_yaw), "chain %d: d_pitch_yaw not finite", i);
        a->ch[i].d = float(c.d_pitch_yaw);
        for (int j = 0; j < 3; j++) {
            TK_REQUIRE(c.q_ub[j] > c.q_lb[j], "chain %d: joint %d has q_ub <= q_lb", i, j);
            a->ch[i].lb[j] = float(c.q_lb[j]);
            a->ch[i].ub[j] = float(c.q_ub[j]);
        }
        for (int j = 0; j < 4; j++) {
            TK_REQUIRE(c.keypoints[j][3] >= 0 && c.keypoints[j][3] <= 3 &&
                           c.keypoints[j][3] == double(int(c.keypoints[j][3])),
                       "chain %d: keypoint %d has invalid link id", i, j);
            for (int e = 0; e < 3; e++) a->ch[i].kp[j][e] = float(c.keypoints[j][e]);
            a->ch[i].kp_link[j] = int(c.keypoints[j][3]);
        }
    }
    a->n_arms = n_arms;
    return TK_OK;
}

tk_status make_loss_args(int32_t batch, int32_t kind, double lambda_app, const float* d_kp, const float* d_kp_ref,
                         int32_t n_arms, double lambda_kp, double tau, LossArgs* la) {
    TK_REQUIRE((kind & ~TK_KP_TWO_TIPS) == 0 || (kind & ~TK_KP_TWO_TIPS) == 1,
               "kind = %d must be 0 (1 - IoU) or 1 (render loss), optionally | TK_KP_TWO_TIPS", kind);
    TK_REQUIRE(std::isfinite(lambda_app) && std::isfinite(lambda_kp) && std::isfinite(tau), "non-finite weights");
    TK_REQUIRE((d_kp == nullptr) == (d_kp_ref == nullptr), "kp and kp_ref must both be given or both NULL");
    TK_REQUIRE(d_kp == nullptr || (n_arms >= 1 && n_arms <= kMaxArms), "n_arms = %d outside 1..%d", n_arms,
               kMaxArms);
    *la = LossArgs{lambda_app, lambda_kp, tau, batch, kind, n_arms};
    return TK_OK;
}

tk_status validate_meshes(const tk_mesh* meshes, int32_t n_meshes, MeshSet* out) {
    TK_REQUIRE(meshes != nullptr, "meshes is NULL");
    TK_REQUIRE(n_meshes >= 1 && n_meshes <= kMaxArms, "n_meshes = %d outside 1..%d", n_meshes, kMaxArms);
    int64_t total = 0;
    out->n_meshes = n_meshes;
    for (int i = 0; i < n_meshes; i++) {
        const tk_mesh& m = meshes[i];
        TK_REQUIRE(m.n_vertices >= 1 && m.n_vertices <= (1 << 24), "mesh %d: n_vertices = %d", i, m.n_vertices);
        TK_REQUIRE(m.n_triangles >= 0 && m.n_triangles <= (1 << 24), "mesh %d: n_triangles = %d", i,
                   m.n_triangles);
        TK_REQUIRE(m.vertices != nullptr && m.vertex_link != nullptr, "mesh %d: NULL vertex arrays", i);
        TK_REQUIRE(m.n_triangles == 0 || m.triangles != nullptr, "mesh %d: NULL triangles", i);
        TK_REQUIRE((reinterpret_cast<uintptr_t>(m.vertices) & 3) == 0 &&
                       (reinterpret_cast<uintptr_t>(m.triangles) & 3) == 0,
                   "mesh %d: misaligned arrays", i);
        out->m[i].vertices = m.vertices;
        out->m[i].triangles = m.triangles;
        out->m[i].vertex_link = m.vertex_link;
        out->m[i].n_vertices = m.n_vertices;
        out->m[i].n_triangles = m.n_triangles;
        out->m[i].vertex_offset = static_cast<int32_t>(total);
        TK_REQUIRE(m.closed == 0 || m.closed == 1, "mesh %d: closed = %d must be 0 or 1", i, m.closed);
        out->m[i].closed = m.closed;
        total += m.n_vertices;
    }
    for (int i = n_meshes; i < kMaxArms; i++) out->m[i] = MeshK{nullptr, nullptr, nullptr, 0, 0, 0, 0};
    TK_REQUIRE(total <= (1 << 24), "too many vertices in total");
    out->total_vertices = static_cast<int32_t>(total);
    return TK_OK;
}

}  // namespace tk

extern "C" {

const char* tk_status_string(tk_status s) {
    switch (s) {
        case TK_OK: return "TK_OK";
        case TK_ERR_INVALID_ARGUMENT: return "TK_ERR_INVALID_ARGUMENT";
        case TK_ERR_UNSUPPORTED: return "TK_ERR_UNSUPPORTED";
        case TK_ERR_WORKSPACE_TOO_SMALL: return "TK_ERR_WORKSPACE_TOO_SMALL";
        case TK_ERR_DEVICE: return "TK_ERR_DEVICE";
    }
    return "TK_ERR_UNKNOWN";
}

const char* tk_last_error(void) { return tk::g_last_error.c_str(); }

int32_t tk_version(void) { return 100; }

}  // extern "C"
