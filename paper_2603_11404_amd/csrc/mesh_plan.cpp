// Host-side claim order of a mesh's triangle chunks for the rasteriser.
//
// The raster kernel takes triangles in chunks of 64, one per lane, and its
// waves claim chunks in index order.  Chunk costs differ by an order of
// magnitude (large faces queue many pixel tasks), and the kernel ends when its
// slowest wave does, so the costly chunks should be claimed first: the waves
// then finish on cheap chunks and end close together (longest-first list
// scheduling).  Sorting the whole blocks, rather than single triangles, keeps
// the vertex locality of each chunk.
//
// The cost of a block is estimated by the summed model-space area of its
// triangles: rigid link motion preserves it and the camera scales every area
// alike, so the order needs neither a pose nor a camera.  Blocks are cut from
// the end of the list, so the one short block (n mod 64 triangles) holds the
// first triangles and goes last: only the last chunk of a mesh may be short.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "tk_internal.h"

using namespace tk;

namespace {
constexpr int32_t kChunk = 64;           // triangles per chunk of the raster kernel (one per lane of a wave)
constexpr int32_t kMaxMesh = 1 << 24;    // mesh size limit of the raster entry points
}  // namespace

extern "C" tk_status tk_mesh_chunk_order(const float* vertices, int32_t n_vertices, const int32_t* triangles,
                                         int32_t n_triangles, int32_t* triangles_out) {
    clear_error();
    TK_REQUIRE(n_vertices >= 1 && n_vertices <= kMaxMesh, "n_vertices %d outside 1..%d", n_vertices,
               kMaxMesh);
    TK_REQUIRE(n_triangles >= 0 && n_triangles <= kMaxMesh, "n_triangles %d outside 0..%d", n_triangles,
               kMaxMesh);
    if (n_triangles == 0) return TK_OK;
    TK_REQUIRE(vertices != nullptr && triangles != nullptr && triangles_out != nullptr, "NULL pointer");
    const uintptr_t in0 = reinterpret_cast<uintptr_t>(triangles), out0 = reinterpret_cast<uintptr_t>(triangles_out);
    const uintptr_t bytes = 3 * sizeof(int32_t) * uintptr_t(n_triangles);
    TK_REQUIRE(out0 + bytes <= in0 || in0 + bytes <= out0, "triangles_out overlaps triangles");
    for (size_t i = 0; i < 3 * size_t(n_triangles); i++)
        TK_REQUIRE(triangles[i] >= 0 && triangles[i] < n_vertices, "triangle %zu: vertex index %d outside 0..%d",
                   i / 3, triangles[i], n_vertices - 1);

    const int32_t head = n_triangles % kChunk;               // the short block: triangles [0, head)
    const int32_t full = (n_triangles - head) / kChunk;      // block k: [head + 64 k, head + 64 (k + 1))
    std::vector<double> cost(full, 0.0);
    for (int32_t k = 0; k < full; k++) {
        double sum = 0.0;
        for (int32_t t = head + k * kChunk; t < head + (k + 1) * kChunk; t++) {
            const float* a = vertices + 3 * size_t(triangles[3 * size_t(t)]);
            const float* b = vertices + 3 * size_t(triangles[3 * size_t(t) + 1]);
            const float* c = vertices + 3 * size_t(triangles[3 * size_t(t) + 2]);
            const double u[3] = {double(b[0]) - a[0], double(b[1]) - a[1], double(b[2]) - a[2]};
            const double v[3] = {double(c[0]) - a[0], double(c[1]) - a[1], double(c[2]) - a[2]};
            const double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
            const double area2 = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            sum += area2 == area2 ? area2 : 0.0;   // a non-finite vertex adds nothing
        }
        cost[k] = sum;
    }
    std::vector<int32_t> order(full);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    int32_t* out = triangles_out;
    for (int32_t k : order) {
        std::copy(triangles + 3 * size_t(head + k * kChunk), triangles + 3 * size_t(head + (k + 1) * kChunk), out);
        out += 3 * size_t(kChunk);
    }
    std::copy(triangles, triangles + 3 * size_t(head), out);
    return TK_OK;
}

// ---------------------------------------------------------------- closed surfaces

// A triangle list is a closed, consistently oriented surface (a 2-cycle) when
// every directed edge a->b occurs as often as b->a.  Counted over sorted
// edge keys: each triangle contributes its three directed edges.
extern "C" tk_status tk_mesh_closed(const int32_t* triangles, int32_t n_triangles, int32_t n_vertices,
                                    int32_t* closed) {
    clear_error();
    TK_REQUIRE(closed != nullptr, "closed is NULL");
    TK_REQUIRE(n_vertices >= 1 && n_vertices <= kMaxMesh, "n_vertices %d outside 1..%d", n_vertices, kMaxMesh);
    TK_REQUIRE(n_triangles >= 0 && n_triangles <= kMaxMesh, "n_triangles %d outside 0..%d", n_triangles,
               kMaxMesh);
    TK_REQUIRE(n_triangles == 0 || triangles != nullptr, "triangles is NULL");
    for (size_t i = 0; i < 3 * size_t(n_triangles); i++)
        TK_REQUIRE(triangles[i] >= 0 && triangles[i] < n_vertices, "triangle %zu: vertex index %d outside 0..%d",
                   i / 3, triangles[i], n_vertices - 1);
    // forward edges a->b as (a, b) and reversed ones as (b, a) with a tag, so
    // that equal undirected edges sort together and the two directions count apart
    std::vector<uint64_t> fwd, rev;
    fwd.reserve(3 * size_t(n_triangles));
    rev.reserve(3 * size_t(n_triangles));
    for (int32_t t = 0; t < n_triangles; t++)
        for (int e = 0; e < 3; e++) {
            const uint64_t a = uint32_t(triangles[3 * size_t(t) + e]);
            const uint64_t b = uint32_t(triangles[3 * size_t(t) + (e + 1) % 3]);
            if (a == b) continue;                    // a repeated vertex: the edge and its reverse coincide
            if (a < b) fwd.push_back(a << 32 | b);
            else rev.push_back(b << 32 | a);
        }
    std::sort(fwd.begin(), fwd.end());
    std::sort(rev.begin(), rev.end());
    *closed = fwd == rev ? 1 : 0;
    return TK_OK;
}

// ---------------------------------------------------------------- plane order

// Triangles sorted by their supporting plane in model space: link of the first
// vertex, then the direction of the unit normal (polar band of 2 degrees, then
// azimuth in 0.01-degree bins), then the plane's offset along it (0.1 um
// bins); equal keys keep list order.  The
// projected orientation of coplanar triangles of one link agrees for every
// pose (it is the side of the plane the camera is on), so 64-triangle chunks
// cut from this order are mostly wholly front- or back-facing, which lets the
// one-sided rasteriser skip whole back-facing chunks.
extern "C" tk_status tk_mesh_plane_order(const float* vertices, const uint8_t* vertex_link, int32_t n_vertices,
                                         const int32_t* triangles, int32_t n_triangles, int32_t* triangles_out) {
    clear_error();
    TK_REQUIRE(n_vertices >= 1 && n_vertices <= kMaxMesh, "n_vertices %d outside 1..%d", n_vertices, kMaxMesh);
    TK_REQUIRE(n_triangles >= 0 && n_triangles <= kMaxMesh, "n_triangles %d outside 0..%d", n_triangles,
               kMaxMesh);
    if (n_triangles == 0) return TK_OK;
    TK_REQUIRE(vertices != nullptr && vertex_link != nullptr && triangles != nullptr && triangles_out != nullptr,
               "NULL pointer");
    const uintptr_t in0 = reinterpret_cast<uintptr_t>(triangles), out0 = reinterpret_cast<uintptr_t>(triangles_out);
    const uintptr_t bytes = 3 * sizeof(int32_t) * uintptr_t(n_triangles);
    TK_REQUIRE(out0 + bytes <= in0 || in0 + bytes <= out0, "triangles_out overlaps triangles");
    for (size_t i = 0; i < 3 * size_t(n_triangles); i++)
        TK_REQUIRE(triangles[i] >= 0 && triangles[i] < n_vertices, "triangle %zu: vertex index %d outside 0..%d",
                   i / 3, triangles[i], n_vertices - 1);
    struct Key {
        int32_t link, band;
        int64_t azimuth, offset;   // 0.01-degree bins, 0.1-micrometre bins
    };
    std::vector<Key> key(n_triangles);
    constexpr double kPi = 3.14159265358979323846;
    for (int32_t t = 0; t < n_triangles; t++) {
        const int32_t* tri = triangles + 3 * size_t(t);
        const float* a = vertices + 3 * size_t(tri[0]);
        const float* b = vertices + 3 * size_t(tri[1]);
        const float* c = vertices + 3 * size_t(tri[2]);
        const double u[3] = {double(b[0]) - a[0], double(b[1]) - a[1], double(b[2]) - a[2]};
        const double v[3] = {double(c[0]) - a[0], double(c[1]) - a[1], double(c[2]) - a[2]};
        double n[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        Key k{int32_t(vertex_link[tri[0]]), 1 << 30, 0, 0};   // degenerate or non-finite: last in its link
        if (len > 0.0 && std::isfinite(len)) {
            for (double& x : n) x /= len;
            const double polar = std::acos(std::min(1.0, std::max(-1.0, n[2])));
            k.band = int32_t(std::floor(polar * (90.0 / kPi)));   // 2-degree bands
            k.azimuth = int64_t(std::floor(std::atan2(n[1], n[0]) * (18000.0 / kPi)));
            k.offset = int64_t(std::floor((n[0] * a[0] + n[1] * a[1] + n[2] * a[2]) * 1e7));
        }
        key[t] = k;
    }
    std::vector<int32_t> order(n_triangles);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        const Key &p = key[x], &q = key[y];
        if (p.link != q.link) return p.link < q.link;
        if (p.band != q.band) return p.band < q.band;
        if (p.azimuth != q.azimuth) return p.azimuth < q.azimuth;
        return p.offset < q.offset;
    });
    for (int32_t i = 0; i < n_triangles; i++)
        std::copy(triangles + 3 * size_t(order[i]), triangles + 3 * size_t(order[i]) + 3, triangles_out + 3 * size_t(i));
    return TK_OK;
}
