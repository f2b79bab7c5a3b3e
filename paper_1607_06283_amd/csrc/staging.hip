// Copy kernel for host-built records: pinned host memory -> device memory.
//
// A push from host memory is one packed record of a few kilobytes to a few
// hundred kilobytes, and a batched solve has one such record per camera.  A
// copy engine transfer, ordered between two kernels of the same stream,
// makes the stream hand over from the compute queue to the copy engine and
// back; a kernel that reads the host memory itself keeps the stream on one
// queue, and one launch moves every record pending on the stream.  Row y of
// the grid is copy y; each thread moves 16-byte words, consecutive threads
// consecutive words, so every wavefront reads 1 KiB of contiguous host
// memory per pass.
#include "staging.h"

#include <hip/hip_ext.h>

#include <cstdint>

namespace rec {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kMaxBlocks = 4096;  // per copy (grid-stride beyond)

struct PullList {
    const uint4* src[kMaxPulls];
    uint4* dst[kMaxPulls];
    int64_t n16[kMaxPulls];
};

__global__ void __launch_bounds__(kThreads) k_pull(PullList L) {
    const int q = blockIdx.y;
    const uint4* __restrict__ src = L.src[q];
    uint4* __restrict__ dst = L.dst[q];
    const int64_t n16 = L.n16[q];
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_pulls(const PullDesc* list, int count, hipStream_t stream, hipEvent_t start,
                        hipEvent_t stop) {
    if (count < 1 || count > kMaxPulls) return hipErrorInvalidValue;
    PullList L = {};
    int64_t blocks = 1;
    for (int q = 0; q < count; ++q) {
        const PullDesc& d = list[q];
        if (((uintptr_t)d.src | (uintptr_t)d.dst | d.bytes) & 15) return hipErrorInvalidValue;
        L.src[q] = (const uint4*)d.src;
        L.dst[q] = (uint4*)d.dst;
        L.n16[q] = (int64_t)(d.bytes / 16);
        const int64_t b = (L.n16[q] + kThreads - 1) / kThreads;
        if (b > blocks) blocks = b;
    }
    if (blocks > kMaxBlocks) blocks = kMaxBlocks;
    const dim3 grid((unsigned)blocks, (unsigned)count), block(kThreads);
    if (start || stop)
        hipExtLaunchKernelGGL(k_pull, grid, block, 0, stream, start, stop, 0, L);
    else
        hipLaunchKernelGGL(k_pull, grid, block, 0, stream, L);
    return hipGetLastError();
}

}  // namespace rec
