// Staging of host-pointer event pushes (and of other host-built records):
// the device side of the copy from pinned host memory into the workspace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace rec {

// One copy: `bytes` bytes (a multiple of 16) from `src`, the device address
// of pinned host memory, to `dst` (device memory); both 16-byte aligned, not
// overlapping.
struct PullDesc {
    const void* src;
    void* dst;
    size_t bytes;
};

constexpr int kMaxPulls = 64;  // copies per launch

// Enqueues on `stream` one kernel that performs the `count` copies of
// `list` (1 <= count <= kMaxPulls; the list is passed by value in the
// launch).  The kernel reads the host memory over the bus itself, so the
// copies stay on the stream's compute queue instead of handing it over to
// a copy engine and back.  start / stop (may be null): timing events that
// the launch packet records around the kernel.  hipErrorInvalidValue for a
// count out of range or a misaligned copy.
hipError_t launch_pulls(const PullDesc* list, int count, hipStream_t stream,
                        hipEvent_t start = nullptr, hipEvent_t stop = nullptr);

}  // namespace rec
