// Bandwidth microbenchmarks that measure the roofline denominators of the
// raster kernel on the device it runs on: HBM (a streaming copy) and LDS
// (a loop of conflict-free 128-bit LDS reads and writes).  Measurement only;
// not on the fitness path.
#include "tk_internal.h"

namespace tk {
namespace {

// Grid-stride copy of n16 16-byte words: every byte is read once and written
// once, with 16-byte vector accesses.  Of the shapes tried on MI355X (1, 2, 4
// or 8 words in flight per thread, plain or non-temporal, 1k to 64k
// workgroups), one word per thread over 4 workgroups per CU streamed fastest.
__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                   size_t n16) {
    const size_t stride = size_t(gridDim.x) * blockDim.x;
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// Each of the 4 waves of a workgroup streams 128-bit reads and writes through
// its own 16 KB of LDS: lane l touches consecutive 16-byte words (a wave
// covers 1 KB per access, no bank conflicts).  Per iteration a lane reads 4 and
// writes 4 words; the values feed a running XOR so nothing is elided, and
// lane 0 of each workgroup stores it.  Bytes moved per workgroup:
// iters * 256 threads * 8 accesses * 16 bytes.
constexpr int kLdsWords = 4096;   // 64 KB of uint4 per workgroup
__global__ __launch_bounds__(256) void lds_kernel(int iters, uint32_t* __restrict__ out) {
    __shared__ uint4 s[kLdsWords];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    uint4* w = s + wave * 1024;
    for (int k = lane; k < 1024; k += 64) w[k] = make_uint4(k, k + tid, k ^ tid, 7u);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (int it = 0; it < iters; it++) {
        const int base = (it & 3) * 256;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint4 v = w[base + r * 64 + lane];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
#pragma unroll
        for (int r = 0; r < 4; r++) w[((base + 512) & 1023) + r * 64 + lane] = make_uint4(acc.x + r, acc.y, acc.z, acc.w);
    }
    acc.x ^= acc.y ^ acc.z ^ acc.w;
    for (int off = 32; off > 0; off >>= 1) acc.x ^= __shfl_xor(acc.x, off);
    if (lane == 0) atomicXor(out + blockIdx.x, acc.x);
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

tk_status tk_bench_copy(const void* d_src, void* d_dst, size_t bytes, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_src != nullptr && d_dst != nullptr, "src / dst is NULL");
    TK_REQUIRE(bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(d_src) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(d_dst) & 15) == 0,
               "bytes and pointers must be multiples of 16");
    if (bytes == 0) return TK_OK;
    const int blocks = 256 * 4;   // 4 workgroups per CU
    hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(s),
                       static_cast<const uint4*>(d_src), static_cast<uint4*>(d_dst), bytes / 16);
    return check_launch("tk_bench_copy");
}

tk_status tk_bench_lds(int32_t workgroups, int32_t iters, uint32_t* d_out, tk_stream s) {
    clear_error();
    TK_REQUIRE(d_out != nullptr, "out is NULL");
    TK_REQUIRE(workgroups >= 1 && workgroups <= (1 << 20) && iters >= 1 && iters <= (1 << 24),
               "workgroups = %d, iters = %d out of range", workgroups, iters);
    hipLaunchKernelGGL(lds_kernel, dim3(workgroups), dim3(256), 0, reinterpret_cast<hipStream_t>(s), iters, d_out);
    return check_launch("tk_bench_lds");
}

}  // extern "C"
