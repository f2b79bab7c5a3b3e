// Copy kernel for host-pointer pushes: pinned host memory -> staging ring.
//
// A push from host memory is one packed record of a few kilobytes to a few
// hundred kilobytes.  A copy engine transfer of it, ordered between two
// kernels of the same stream, makes the stream hand over from the compute
// queue to the copy engine and back; a kernel that reads the host memory
// itself keeps the stream on one queue.  Each thread moves 16-byte words,
// consecutive threads consecutive words, so every wavefront reads 1 KiB of
// contiguous host memory per pass.
#include "staging.h"

#include <hip/hip_ext.h>

#include <cstdint>

namespace rec {
namespace {

constexpr int kThreads = 256;
constexpr int64_t kMaxBlocks = 4096;

__global__ void __launch_bounds__(kThreads)
k_pull(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

}  // namespace

hipError_t launch_pull(const void* src, void* dst, size_t bytes, hipStream_t stream,
                       hipEvent_t start, hipEvent_t stop) {
    if (((uintptr_t)src | (uintptr_t)dst | bytes) & 15) return hipErrorInvalidValue;
    if (bytes == 0) return hipSuccess;
    const int64_t n16 = (int64_t)(bytes / 16);
    int64_t blocks = (n16 + kThreads - 1) / kThreads;
    if (blocks > kMaxBlocks) blocks = kMaxBlocks;
    const dim3 grid((unsigned)blocks), block(kThreads);
    if (start || stop)
        hipExtLaunchKernelGGL(k_pull, grid, block, 0, stream, start, stop, 0, (const uint4*)src,
                              (uint4*)dst, n16);
    else
        hipLaunchKernelGGL(k_pull, grid, block, 0, stream, (const uint4*)src, (uint4*)dst, n16);
    return hipGetLastError();
}

}  // namespace rec
