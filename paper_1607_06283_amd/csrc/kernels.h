// Internal interface between the C ABI (rec_api.hip) and the device kernels
// (kernels.hip).  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rec {

constexpr int64_t kNever = INT64_MIN;   // t_last of a pixel that never fired
constexpr int64_t kNoBad = INT64_MAX;   // no rejected event in the current push

// Error codes stored by device-side validation (same values as REC_E*).
constexpr int32_t kErrInval = -1;
constexpr int32_t kErrRange = -2;
constexpr int32_t kErrOrder = -3;

// Device-resident stream state (first 256 bytes of the workspace).
struct alignas(256) DevState {
    int64_t t_ref;          // timestamp of the last accepted event
    int64_t t_first;        // first accepted timestamp of the stream
    int64_t first_bad;      // index of the first invalid event of the running push
    int64_t batch_events;   // events accepted since the last solve
    int64_t last_events;    // events consumed by the last solve
    int32_t started;        // 1 once an event was accepted
    int32_t err;            // first deferred push error not yet reported (0 = none)
};

// Device pointers carved from the caller's workspace.
struct Planes {
    DevState* st;
    float* u[2];            // primal image, ping-pong
    float* p[2];            // dual field, 3 consecutive planes, ping-pong
    float* f;               // data image of the current block
    float* tx;              // forward differences of the time surface
    float* ty;
    int64_t* t_last;        // latest timestamp per pixel (kNever if none)
    int32_t* npos;          // pending event counts
    int32_t* nneg;
    int64_t* ev_t;          // staging for host-pointer pushes
    uint16_t* ev_x;
    uint16_t* ev_y;
    int8_t* ev_p;
    double* gap_part;       // per-block (gap, energy) partial sums
    double* gap_hist;       // (gap, energy) per sample of the running solve
};

struct Frame {
    int32_t W, H;
};

// FP32 constants of the iteration.
struct IterConsts {
    float tau, sigma, taulam, umin, umax;
};

constexpr int kGapBlock = 256;
constexpr int kGapHistCap = 4096;
constexpr int kSmallPush = 32768;  // pushes up to this size use one workgroup

size_t gap_blocks(size_t np);

// Launchers: return the first HIP error (launch errors only; no sync).
hipError_t launch_init(const Planes& P, Frame fr, float u_init, bool keep_u, hipStream_t s);
hipError_t launch_push(const Planes& P, Frame fr, const int64_t* t, const uint16_t* x,
                       const uint16_t* y, const int8_t* pol, int64_t n, hipStream_t s);
hipError_t launch_build(const Planes& P, Frame fr, int cur, double dpos, double dneg,
                        double time_unit_us, hipStream_t s);
hipError_t launch_pd_plain(const Planes& P, Frame fr, IterConsts k, int cur, hipStream_t s);
hipError_t launch_pd_fused(const Planes& P, Frame fr, IterConsts k, int cur, int iters,
                           int rows, int waves, hipStream_t s);
bool fused_shape_supported(int rows, int waves);
hipError_t launch_gap(const Planes& P, Frame fr, double lambda, double umin, double umax,
                      int cur, int slot, hipStream_t s);
hipError_t launch_time_plane(const Planes& P, Frame fr, double time_unit_us, float* out,
                             hipStream_t s);
hipError_t launch_metric_plane(const Planes& P, Frame fr, float* out, hipStream_t s);

}  // namespace rec
