// Staging of host-pointer event pushes: the device side of the copy from
// pinned host memory into the workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace rec {

// Enqueues on `stream` a kernel that copies `bytes` bytes (a multiple of
// 16) from `src`, the device address of pinned host memory, to `dst`
// (device memory); both 16-byte aligned, not overlapping.  The kernel reads
// the host memory over the bus itself, so the copy stays on the stream's
// compute queue.  start / stop (may be null): timing events that the launch
// packet records around the kernel.  hipErrorInvalidValue for a misaligned
// argument.
hipError_t launch_pull(const void* src, void* dst, size_t bytes, hipStream_t stream,
                       hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

}  // namespace rec
