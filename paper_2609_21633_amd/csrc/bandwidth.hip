// Plain streaming device copy: the practical HBM roof that the operator
// kernels are measured against, and the known-size kernel that scales the
// HBM counters (FETCH_SIZE, WRITE_SIZE) of a profile.
#include <cstdint>

#include "tng_internal.hpp"

namespace tng {
namespace {

constexpr int COPY_BLOCK = 256;
constexpr int COPY_UNROLL = 4;

// Each thread moves COPY_UNROLL 16-byte vectors per trip, the loads of a trip
// issued before its stores; consecutive lanes touch consecutive vectors.
__global__ void __launch_bounds__(COPY_BLOCK) stream_copy_kernel(const uint4* __restrict__ src,
                                                                 uint4* __restrict__ dst, long long n) {
    const long long stride = (long long)gridDim.x * COPY_BLOCK * COPY_UNROLL;
    long long i = (long long)blockIdx.x * COPY_BLOCK * COPY_UNROLL + threadIdx.x;
    for (; i + (COPY_UNROLL - 1) * COPY_BLOCK < n; i += stride) {
        uint4 v[COPY_UNROLL];
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) v[u] = src[i + u * COPY_BLOCK];
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) dst[i + u * COPY_BLOCK] = v[u];
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u)
        if (i + u * COPY_BLOCK < n) dst[i + u * COPY_BLOCK] = src[i + u * COPY_BLOCK];
}

}  // namespace

void launch_stream_copy(const tng_ctx* ctx, const void* src, void* dst, size_t bytes) {
    const long long n = (long long)(bytes / sizeof(uint4));
    // enough workgroups to keep every CU's memory pipeline full, a few trips each
    const long long per_block = (long long)COPY_BLOCK * COPY_UNROLL;
    long long blocks = (n + per_block - 1) / per_block;
    const long long cap = (long long)ctx->n_cu * 32;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    ScopedKernelTimer timer(ctx, "stream_copy");
    stream_copy_kernel<<<(unsigned)blocks, COPY_BLOCK, 0, ctx->stream>>>(static_cast<const uint4*>(src),
                                                                         static_cast<uint4*>(dst), n);
    TNG_HIP(hipGetLastError());
}

}  // namespace tng
