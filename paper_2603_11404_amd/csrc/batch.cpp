// Batched independent problems: table layout and the C entry points.
//
// Table (written on the host by tk_batch_describe, used from device memory):
//   [n raster entries][pad to 256 bytes][n update entries][pad to 256 bytes]
//   [control: one int32 pair per persistent launch of up to 128 problems,
//    zero between launches]
#include <cstring>

#include "tk_internal.h"

namespace tk {
namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t update_offset(int32_t n) { return align256(size_t(n) * batch_raster_entry_bytes()); }

size_t control_offset(int32_t n) { return align256(update_offset(n) + size_t(n) * batch_update_entry_bytes()); }

size_t control_bytes(int32_t n) { return align256(size_t(8) * ((n + kMaxBatch - 1) / kMaxBatch)); }

tk_status check_batch(const tk_problem* problems, int32_t n_problems, const void* table) {
    TK_REQUIRE(problems != nullptr, "problems is NULL");
    TK_REQUIRE(n_problems >= 1 && n_problems <= 65536, "n_problems = %d outside 1..65536", n_problems);
    TK_REQUIRE(table != nullptr && (reinterpret_cast<uintptr_t>(table) & 255) == 0,
               "table must be a 256-byte aligned pointer");
    return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

size_t tk_batch_table_bytes(int32_t n_problems) {
    if (n_problems < 1 || n_problems > 65536) return 0;
    return control_offset(n_problems) + control_bytes(n_problems);
}

tk_status tk_batch_describe(const tk_problem* problems, int32_t n_problems, void* h_table, size_t table_bytes) {
    clear_error();
    if (tk_status st = check_batch(problems, n_problems, h_table)) return st;
    const size_t need = tk_batch_table_bytes(n_problems);
    if (table_bytes < need)
        return fail(TK_ERR_WORKSPACE_TOO_SMALL, "tk_batch_describe: table of %zu bytes, %zu needed", table_bytes, need);
    std::memset(h_table, 0, need);
    char* base = static_cast<char*>(h_table);
    for (int i = 0; i < n_problems; i++) {
        if (tk_status st = batch_describe_raster(problems[i], base + size_t(i) * batch_raster_entry_bytes())) {
            const std::string detail = tk_last_error();
            return fail(st, "problem %d: %s", i, detail.c_str());
        }
        if (tk_status st = batch_describe_update(problems[i], base + update_offset(n_problems) +
                                                                 size_t(i) * batch_update_entry_bytes())) {
            const std::string detail = tk_last_error();
            return fail(st, "problem %d: %s", i, detail.c_str());
        }
    }
    return TK_OK;
}

tk_status tk_batch_ask_eval(const tk_problem* problems, int32_t n_problems, const void* d_table, tk_stream s) {
    clear_error();
    if (tk_status st = check_batch(problems, n_problems, d_table)) return st;
    return batch_launch_raster(problems, n_problems, d_table, reinterpret_cast<hipStream_t>(s));
}

tk_status tk_batch_ask_eval_persistent(const tk_problem* problems, int32_t n_problems, void* d_table, tk_stream s) {
    clear_error();
    if (tk_status st = check_batch(problems, n_problems, d_table)) return st;
    int32_t* counters = reinterpret_cast<int32_t*>(static_cast<char*>(d_table) + control_offset(n_problems));
    return batch_launch_persistent(problems, n_problems, d_table, counters, reinterpret_cast<hipStream_t>(s));
}

tk_status tk_batch_tell(const tk_problem* problems, int32_t n_problems, const void* d_table, tk_stream s) {
    clear_error();
    if (tk_status st = check_batch(problems, n_problems, d_table)) return st;
    const char* upd = static_cast<const char*>(d_table) + update_offset(n_problems);
    return batch_launch_tell(problems, n_problems, upd, reinterpret_cast<hipStream_t>(s));
}

}  // extern "C"
